"""Independent references used to pin the oracle (and to check GPU output).

Nothing here imports the oracle or the HIP library.  Each function restates
the *definition* of the result the paper's method reaches, not the method:

* ``bfs_label`` -- brute-force flood fill in linear order.  Clusters are the
  connected components of the face-adjacency graph on occupied sites
  (periodic axes wrap); the cluster met first in linear order (x fastest) is
  number 1, the next new one number 2, ...  This is the numbering the serial
  HK pass with compaction produces (Sec. 2), written without HK.
* ``scipy_label`` -- the library routine ``scipy.ndimage.label`` with the
  6-neighbour structure, plus a separate merge of wrap-around pairs and a
  renumbering by first occurrence.
* ``check_invariants`` -- properties every correct output has at any size.
"""
from __future__ import annotations

from collections import deque

import numpy as np


def occupied(phi):
    """phi > 0 as an IEEE float32 comparison (Sec. 2 condition)."""
    return np.asarray(phi, dtype=np.float32) > np.float32(0)


def bfs_label(phi, mask):
    """Pure-Python breadth-first flood fill (tiny lattices only)."""
    occ = occupied(phi)
    nz, ny, nx = occ.shape
    per = (bool(mask & 1), bool(mask & 2), bool(mask & 4))
    n = (nx, ny, nz)
    flat = occ.ravel().tolist()
    lab = [0] * len(flat)
    sizes = []

    def neighbours(i):
        x = i % nx
        y = (i // nx) % ny
        z = i // (nx * ny)
        c = [x, y, z]
        strides = (1, nx, nx * ny)
        for a in range(3):
            for d in (-1, 1):
                v = c[a] + d
                if v < 0 or v >= n[a]:
                    if not per[a]:
                        continue
                    v %= n[a]
                yield i + (v - c[a]) * strides[a]

    k = 0
    for s in range(len(flat)):
        if not flat[s] or lab[s]:
            continue
        k += 1
        lab[s] = k
        cnt = 0
        q = deque([s])
        while q:
            i = q.popleft()
            cnt += 1
            for j in neighbours(i):
                if flat[j] and not lab[j]:
                    lab[j] = k
                    q.append(j)
        sizes.append(cnt)
    return np.array(lab, dtype=np.int32).reshape(occ.shape), k, np.array(sizes, dtype=np.int64)


def _find(par, a):
    while par[a] != a:
        par[a] = par[par[a]]
        a = par[a]
    return a


def scipy_label(phi, mask):
    """scipy.ndimage.label (6-neighbour) + wrap merge + first-occurrence
    renumbering."""
    from scipy import ndimage

    occ = occupied(phi)
    st = ndimage.generate_binary_structure(3, 1)
    lab, m = ndimage.label(occ, structure=st)
    par = list(range(m + 1))
    nz, ny, nx = occ.shape
    pairs = []
    if (mask & 1) and nx >= 2:
        pairs.append((lab[:, :, 0], lab[:, :, nx - 1]))
    if (mask & 2) and ny >= 2:
        pairs.append((lab[:, 0, :], lab[:, ny - 1, :]))
    if (mask & 4) and nz >= 2:
        pairs.append((lab[0, :, :], lab[nz - 1, :, :]))
    for a, b in pairs:
        sel = (a > 0) & (b > 0)
        for u, v in set(zip(a[sel].tolist(), b[sel].tolist())):
            ru, rv = _find(par, u), _find(par, v)
            if ru != rv:
                par[max(ru, rv)] = min(ru, rv)
    root = np.array([_find(par, i) for i in range(m + 1)], dtype=np.int64)
    cls = root[lab].ravel()
    occf = occ.ravel()
    out = np.zeros(cls.shape, dtype=np.int32)
    if occf.any():
        ids, first = np.unique(cls[occf], return_index=True)
        order = np.argsort(first)            # classes by first occurrence
        rank = np.empty(root.max() + 1, dtype=np.int64)
        rank[ids[order]] = np.arange(1, ids.size + 1)
        out[occf] = rank[cls[occf]]
        k = ids.size
    else:
        k = 0
    sizes = np.bincount(out[occf], minlength=k + 1)[1:].astype(np.int64) if k else np.zeros(0, np.int64)
    return out.reshape(occ.shape), k, sizes


def component_count(phi, mask):
    """Number of connected components (scipy + wrap merge)."""
    return scipy_label(phi, mask)[1]


def check_invariants(phi, mask, labels, k, sizes, check_connected=True):
    """Raise AssertionError unless (labels, k, sizes) satisfies every
    property of a correct canonical labelling."""
    occ = occupied(phi)
    labels = np.asarray(labels)
    sizes = np.asarray(sizes)
    assert labels.shape == occ.shape
    assert labels.dtype == np.int32
    # medium <-> label 0
    assert np.array_equal(labels == 0, ~occ), "label 0 must mark exactly the medium"
    n = occ.size
    assert 0 <= k <= (n + 1) // 2, "K exceeds the V/2 bound"
    assert sizes.shape == (k,)
    if k == 0:
        assert not occ.any()
        return
    assert labels.min() >= 0 and labels.max() == k
    # sizes by counting
    cnt = np.bincount(labels.ravel(), minlength=k + 1)[1:]
    assert np.array_equal(cnt, sizes), "sizes disagree with label counts"
    assert sizes.min() >= 1 and int(sizes.sum()) == int(occ.sum())
    # face-adjacent occupied pairs share a label (no two clusters touch)
    nz, ny, nx = occ.shape
    for axis, bit, length in ((2, 1, nx), (1, 2, ny), (0, 4, nz)):
        if length >= 2:
            a = np.take(labels, range(0, length - 1), axis=axis)
            b = np.take(labels, range(1, length), axis=axis)
            both = (a > 0) & (b > 0)
            assert np.array_equal(a[both], b[both]), f"neighbours differ along axis {axis}"
            if mask & bit:
                a = np.take(labels, [length - 1], axis=axis)
                b = np.take(labels, [0], axis=axis)
                both = (a > 0) & (b > 0)
                assert np.array_equal(a[both], b[both]), f"wrap neighbours differ along axis {axis}"
    # canonical: first occurrences in linear order are 1, 2, ..., K
    flat = labels.ravel()
    ids, first = np.unique(flat[flat > 0], return_index=True)
    assert ids.size == k
    order = ids[np.argsort(first)]
    assert np.array_equal(order, np.arange(1, k + 1)), "labels not in first-occurrence order"
    # each label is one connected set: component count equals K
    if check_connected:
        assert component_count(phi, mask) == k, "a label spans several components"

"""Interior/exterior decision of the capsule algorithm: TEST INFRASTRUCTURE ONLY.

Same rules as the rest of ``oracle/``: only ``tests/``, ``smoke()`` and
``bench.py``'s cpu_baseline leg may use it; it imports nothing from the
product.

Sec. 6, last step of the interior-detection algorithm: the HK pass labels
the sites that kept the far-field proximity value I0 (here: ``labels`` > 0,
numbered 1..K).  Each such cluster is then judged by the proximity values I
of the membrane sites that border it -- an interior pocket is surrounded by
negative values, the exterior by positive ones.  Written out:

* a border pair is a face-adjacent pair (s, j) of a cluster site s and a
  non-cluster site j (labels[j] == 0), with periodic wrap on the axes of the
  mask; an axis of length 1 has no pair, and on a periodic axis of length 2
  the two neighbours coincide and give one pair (the same reading as the
  connectivity of the labelling itself);
* neg[k-1] / pos[k-1] = number of border pairs of cluster k whose I[j] is
  < 0 / > 0 (0 and NaN count for neither side);
* inside[k-1] = 1 if neg > pos, 0 if pos > neg, -1 on a tie (including a
  cluster with no border pair at all).
"""
from __future__ import annotations

import numpy as np


def _neighbour_views(a, axis, n, periodic):
    """(neighbour values, valid mask) for the +1 and -1 neighbours of every
    site along `axis` (array axis), following the pair rules above."""
    out = []
    if n == 1:
        return out
    if periodic:
        shifts = (1,) if n == 2 else (1, -1)
        for sh in shifts:
            out.append((np.roll(a, sh, axis=axis), None))
        return out
    for sh in (1, -1):
        v = np.roll(a, sh, axis=axis)
        valid = np.ones(a.shape, dtype=bool)
        idx = [slice(None)] * a.ndim
        idx[axis] = 0 if sh == 1 else n - 1  # the rolled-in site is not a neighbour
        valid[tuple(idx)] = False
        out.append((v, valid))
    return out


def classify(I, labels, k, periodic):
    """Return (neg, pos, inside) for clusters 1..k; I float32 and labels
    int32, both (nz, ny, nx); periodic = int mask (bit 0 = x) or (px, py, pz)."""
    I = np.asarray(I, dtype=np.float32)
    labels = np.asarray(labels, dtype=np.int32)
    if isinstance(periodic, (int, np.integer)):
        mask = int(periodic)
    else:
        px, py, pz = periodic
        mask = (1 if px else 0) | (2 if py else 0) | (4 if pz else 0)
    neg = np.zeros(k, dtype=np.int64)
    pos = np.zeros(k, dtype=np.int64)
    nz, ny, nx = labels.shape
    # array axis 2 = x (mask bit 0), 1 = y (bit 1), 0 = z (bit 2)
    for axis, n, bit in ((2, nx, 1), (1, ny, 2), (0, nz, 4)):
        per = bool(mask & bit)
        for (nl, valid), (nI, _) in zip(_neighbour_views(labels, axis, n, per),
                                        _neighbour_views(I, axis, n, per)):
            m = (labels > 0) & (nl == 0)
            if valid is not None:
                m &= valid
            lab = labels[m] - 1
            v = nI[m]
            np.add.at(neg, lab, (v < 0).astype(np.int64))
            np.add.at(pos, lab, (v > 0).astype(np.int64))
    inside = np.where(neg > pos, 1, np.where(pos > neg, 0, -1)).astype(np.int8)
    return neg, pos, inside

"""GPU tests that drive each bounded fast structure of the path past its
capacity, so that its exact fallback runs, and check that it ran (the
library's fallback counters, hk_debug_counters) and that the results still
equal the oracle's:

* merge: more distinct face pairs in one brick than its LDS pair list holds
  (the extra pairs are united where found);
* roots: more distinct cluster roots among the nodes of one group of
  bricks than the group's LDS hash holds (sizes added to the root directly);
* write: more component slots and runs in one brick than the write phase's
  LDS holds (run slots read from global memory).

The face pattern: every brick face layer (y or z of a brick boundary, and
x = 0 / 63 of a 64-wide brick) holds a site checkerboard and nothing else
is occupied, so the sites of a face layer are isolated inside their brick
and each one meets exactly one isolated site of the next brick: every
brick has about 1150 distinct face pairs on its low faces (its list holds
1024), and every such pair is a two-site cluster whose root one group of
four bricks must hold in its hash (1024 slots)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1405_1931_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1405_1931_amd as hk

    hk.set_brick(16, 16)
    yield hk
    hk.set_brick(0, 0)


def face_layers(shape, by=16, bz=16):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    occ = (((y % by == 0) | (y % by == by - 1)) & ((x + z) % 2 == 0)) | \
          (((z % bz == 0) | (z % bz == bz - 1)) & ((x + y) % 2 == 0)) | \
          (((x % 64 == 0) | (x % 64 == 63)) & ((y + z) % 2 == 0))
    return np.where(occ, np.float32(1.0), np.float32(-1.0))


def check(hk, phi_np, mask, what):
    print(f"[fallback] {what} {phi_np.shape} mask {mask}", flush=True)
    hk.debug_counters()  # clear
    lab, k, sz = hk.label(torch.from_numpy(phi_np).cuda(), mask)
    counts = hk.debug_counters()
    el, ek, es = oracle.label(phi_np, mask)
    assert k == ek, what
    assert np.array_equal(lab.cpu().numpy(), el), what
    assert np.array_equal(sz.cpu().numpy(), es), what
    assert hk.device_error() == 0
    return counts


@pytest.mark.parametrize("mask", [7, 0, 5])
def test_merge_pair_list_and_roots_hash_overflow(hk, mask):
    counts = check(hk, face_layers((64, 64, 192)), mask, "face layers")
    assert counts["merge_direct"] > 0, counts
    assert counts["roots_direct"] > 0, counts


def test_face_layers_ragged_and_batched(hk):
    """The same overflowing bricks, ragged at the high ends, alone and in
    one batch with other lattices."""
    phi = face_layers((40, 52, 150))
    counts = check(hk, phi, 7, "face layers, ragged")
    assert counts["merge_direct"] > 0, counts
    items = [(phi, 7), (face_layers((64, 48, 128)), 3), (W.percolation((30, 40, 70), 0.4, seed=3), 6)]
    hk.debug_counters()
    out = hk.label_batched([(torch.from_numpy(p).cuda(), m) for p, m in items])
    torch.cuda.synchronize()
    counts = hk.debug_counters()
    assert counts["merge_direct"] > 0 and counts["roots_direct"] > 0, counts
    for j, ((p, m), (lab, k, sz)) in enumerate(zip(items, out)):
        el, ek, es = oracle.label(p, m)
        assert k == ek and np.array_equal(lab.cpu().numpy(), el) and np.array_equal(sz.cpu().numpy(), es), j
    assert hk.device_error() == 0


@pytest.mark.parametrize("mask", [0, 7])
def test_write_runs_from_global_memory(hk, mask):
    """A site checkerboard fills every brick's run table (32 runs per row)
    and has as many components as runs: the run slots do not fit beside the
    slot labels in the write phase's LDS."""
    nz, ny, nx = 48, 32, 128
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phi = np.where((x + y + z) % 2 == 0, np.float32(1.0), np.float32(-1.0))
    counts = check(hk, phi, mask, "site checkerboard")
    assert counts["runs_global"] > 0, counts

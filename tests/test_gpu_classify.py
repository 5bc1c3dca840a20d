"""GPU parity of the interior/exterior decision (Sec. 6, last step): hk_classify
against the oracle, element by element (counts and decisions), on the labels
hk_label produced for the same lattice."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import classify as C
from paper_1405_1931_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1405_1931_amd as hk

    hk.set_brick(0, 0)
    return hk


def cluster_field(I):
    return np.where(I == np.float32(W.I0), np.float32(1), np.float32(-1)).astype(np.float32)


def offset_view(t, off):
    """A copy of t whose data starts `off` elements into its own buffer (so
    its address is not 16-byte aligned for off = 1..3)."""
    buf = torch.empty(t.numel() + off, dtype=t.dtype, device=t.device)
    v = buf[off:].view(t.shape)
    v.copy_(t)
    return v


def check(hk, I_np, mask, what, off=0):
    print(f"[classify] {what} {I_np.shape} mask {mask} offset {off}", flush=True)
    I = offset_view(torch.from_numpy(np.ascontiguousarray(I_np)).cuda(), off)
    phi = torch.from_numpy(cluster_field(I_np)).cuda()
    nz, ny, nx = I.shape
    labels = offset_view(torch.empty_like(phi, dtype=torch.int32), off)
    kbuf = torch.zeros(1, dtype=torch.int64, device="cuda")
    sizes = torch.empty(max(1, hk.max_clusters(nx, ny, nz)), dtype=torch.int64, device="cuda")
    hk.label_into(phi, mask, labels, kbuf, sizes)
    neg, pos, inside = hk.classify(I, labels, kbuf, mask)
    k = int(kbuf.item())
    en, ep, ei = C.classify(I_np, labels.cpu().numpy(), k, mask)
    assert np.array_equal(neg.cpu().numpy(), en), what
    assert np.array_equal(pos.cpu().numpy(), ep), what
    assert np.array_equal(inside.cpu().numpy(), ei), what
    return k, ei


def test_hand_worked_fixtures(hk):
    from test_classify_pins import load_fixture

    for name in ("plane_ring.txt", "row_ties.txt"):
        I, cases = load_fixture(name)
        for case in cases:
            k, ei = check(hk, I, case["mask"], name)
            assert k == case["k"][0] and ei.tolist() == case["inside"]


@pytest.mark.parametrize("shape", [(1, 1, 7), (2, 2, 2), (3, 5, 70), (9, 33, 65), (17, 2, 130), (40, 41, 42)])
def test_random_fields_all_masks(hk, shape):
    rng = np.random.default_rng(sum(shape))
    # values that stress the sign test: +-0, NaN, denormals of both signs
    vals = np.array([W.I0, W.I0, W.I0, -0.3, 0.2, 0.0, -0.0, np.nan,
                     np.float32(1e-42), np.float32(-1e-42), 0.45], dtype=np.float32)
    I = rng.choice(vals, size=shape).astype(np.float32)
    for mask in range(8):
        check(hk, I, mask, f"random {shape}")


@pytest.mark.parametrize("shape", [(3, 4, 4), (5, 6, 8), (7, 9, 260), (2, 3, 512), (4, 1, 12), (1, 2, 4)])
def test_rows_of_four_sites_both_paths(hk, shape):
    """Rows whose length is a multiple of 4 take four sites per lane when the
    arrays are 16-byte aligned and one site per lane when they are not; both
    must equal the oracle."""
    rng = np.random.default_rng(sum(shape) + 1)
    vals = np.array([W.I0, W.I0, W.I0, -0.3, 0.2, 0.0, -0.0, np.nan,
                     np.float32(1e-42), np.float32(-1e-42), 0.45], dtype=np.float32)
    I = rng.choice(vals, size=shape).astype(np.float32)
    for mask in range(8):
        for off in (0, 1):
            check(hk, I, mask, f"rows of 4k sites {shape}", off)


def test_capsules_scaled_and_full(hk):
    for scale in (4, 2, 1):
        phi, I, mask = W.capsule_config(scale)
        assert np.array_equal(cluster_field(I), phi)
        caps = max(1, round(300 / scale ** 3))
        for off in ((0, 3) if scale > 1 else (0,)):
            k, ei = check(hk, I, mask, f"capsules 1/{scale}", off)
            assert k == caps + 1
            assert ei[0] == 0 and np.all(ei[1:] == 1)
    assert hk.device_error() == 0


def test_no_clusters_and_no_border(hk):
    check(hk, np.full((5, 6, 7), 0.3, dtype=np.float32), 7, "no cluster site")
    k, ei = check(hk, np.full((5, 6, 7), W.I0, dtype=np.float32), 7, "one cluster, no border")
    assert k == 1 and ei.tolist() == [-1]

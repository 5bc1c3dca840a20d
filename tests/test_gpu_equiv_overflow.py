"""The brick labelling when a brick's runs and its stored rule-3 equivalences
(Sec. 2) together exceed the brick's run table: the overlaps are then united
again directly, row against row.

Planes of even x, fully occupied, give every 64 x 16 x 16 brick 32
single-site runs in each of its 256 rows (8192 runs: the whole table) and
an equivalence for almost every run (its parent through y - 1, a second
link through z - 1), so every brick takes that path.  With nx even the
planes never touch, also across an x wrap (x = nx - 1 is odd): K = nx / 2,
every size ny * nz, plane x numbered x / 2 + 1.  Ragged lattices, odd nx
under a wrap and stripes with noise are checked against the oracle."""
from __future__ import annotations

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1405_1931_amd as hk

    hk.set_brick(16, 16)  # the brick whose run table the stripes fill
    yield hk
    hk.set_brick(0, 0)


def stripes_np(shape, noise=0.0, seed=0):
    nz, ny, nx = shape
    occ = np.broadcast_to((np.arange(nx) % 2 == 0).reshape(1, 1, -1), shape)
    if noise:
        occ = occ | (np.random.default_rng(seed).random(shape) < noise)
    return np.where(occ, 1.0, -1.0).astype(np.float32)


@pytest.mark.parametrize("mask", [0, 7])
def test_stripes_closed_form(hk, mask):
    for shape in ((64, 64, 256), (128, 96, 1024)):
        print(f"[overflow] x stripes {shape} mask {mask}", flush=True)
        nz, ny, nx = shape
        x = torch.arange(nx, device="cuda", dtype=torch.int32).view(1, 1, nx)
        occ = (x % 2) == 0
        phi = torch.where(occ, 1.0, -1.0).to(torch.float32).expand(nz, ny, nx).contiguous()
        hk.debug_counters()  # clear
        labels, k, sizes = hk.label(phi, mask)
        # every brick took the overflow path (the fallback counter proves it)
        nb = (nx // 64) * (ny // 16) * (nz // 16)
        assert hk.debug_counters()["equiv_again"] == nb
        assert k == nx // 2
        assert bool((sizes == ny * nz).all())
        expect = torch.where(occ, torch.div(x, 2, rounding_mode="floor") + 1, 0).to(torch.int32)
        assert torch.equal(labels, expect.expand(nz, ny, nx))
        assert hk.device_error() == 0


def assert_oracle(hk, phi_np, mask, what):
    print(f"[overflow] {what} shape={phi_np.shape} mask={mask}", flush=True)
    lab, k, s = hk.label(torch.from_numpy(phi_np).cuda(), mask)
    exp = oracle.label(phi_np, mask)
    assert k == exp[1], what
    assert np.array_equal(lab.cpu().numpy(), exp[0]), what
    assert np.array_equal(s.cpu().numpy(), exp[2]), what
    assert hk.device_error() == 0


@pytest.mark.parametrize("shape", [(40, 24, 130), (17, 33, 199), (32, 32, 128)])
def test_stripes_vs_oracle(hk, shape):
    for mask in (0, 1, 6, 7):
        assert_oracle(hk, stripes_np(shape), mask, "x stripes")
    for noise, seed in ((0.02, 1), (0.1, 2)):
        for mask in (0, 7):
            assert_oracle(hk, stripes_np(shape, noise, seed), mask, f"x stripes + {noise} noise")


def test_stripes_batched(hk):
    """The same path in the grouped launches of one batched call."""
    shapes = [(40, 24, 130), (32, 32, 128), (17, 33, 199), (64, 64, 256)]
    items = [(stripes_np(sh, 0.05 * (i % 2), seed=i), (0, 7, 1, 6)[i]) for i, sh in enumerate(shapes)]
    print(f"[overflow] batched x stripes, {len(items)} jobs", flush=True)
    out = hk.label_batched([(torch.from_numpy(p).cuda(), m) for p, m in items])
    torch.cuda.synchronize()
    assert hk.device_error() == 0
    for j, ((p, m), (lab, k, sz)) in enumerate(zip(items, out)):
        exp = oracle.label(p, m)
        assert k == exp[1], f"job {j}"
        assert np.array_equal(lab.cpu().numpy(), exp[0]), f"job {j}"
        assert np.array_equal(sz.cpu().numpy(), exp[2]), f"job {j}"


@pytest.mark.parametrize("mask", [0, 7])
def test_stripes_incremental(hk, mask):
    """The same path for the bricks an incremental call labels anew: every
    call equals the oracle, and only the bricks whose words changed are
    labelled again."""
    shape = (48, 40, 192)  # 3 x 3 x 3 bricks: full along x and z, ragged along y
    nz, ny, nx = shape
    f0 = stripes_np(shape)
    f1 = f0.copy()
    f1[20, 20, 71] = 1.0    # joins planes 70 and 72 inside brick (1, 1, 1)
    f2 = f1.copy()
    f2[0, 0, 1:4] = 1.0     # joins planes 0, 2 and 4 in brick (0, 0, 0)
    with hk.Incremental(shape, mask) as st:
        for f, what, rel in ((f0, "stripes", 27), (f1, "one site joins two planes", 1),
                             (f2, "a short run joins three planes", 1), (f2, "unchanged", 0)):
            print(f"[overflow] incremental {what} mask {mask}", flush=True)
            labels, k, sizes, r = st.label(torch.from_numpy(f).cuda())
            el, ek, es = oracle.label(f, mask)
            assert k == ek, what
            assert np.array_equal(labels.cpu().numpy(), el), what
            assert np.array_equal(sizes.cpu().numpy(), es[:ek]), what
            assert r == rel, (what, r)
            assert st.device_error() == 0

"""GPU parity: hk_label (through the C-ABI) against the serial oracle,
bit for bit on labels, K and sizes (tolerance 0: the result is integer and
unique), plus invariants at every size."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1405_1931_amd import workloads as W
from pins import check_invariants

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1405_1931_amd as hk

    hk.set_brick(0, 0)
    return hk


def gpu_label(hk, phi_np, mask):
    phi = torch.from_numpy(np.ascontiguousarray(phi_np)).cuda()
    lab, k, s = hk.label(phi, mask)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), k, s.cpu().numpy()


def assert_parity(hk, phi_np, mask, what=""):
    print(f"[parity] {what} shape={phi_np.shape} mask={mask}", flush=True)
    got = gpu_label(hk, phi_np, mask)
    exp = oracle.label(phi_np, mask)
    assert got[1] == exp[1], f"{what}: K {got[1]} != {exp[1]}"
    if not np.array_equal(got[0], exp[0]):
        bad = np.argwhere(got[0] != exp[0])
        raise AssertionError(f"{what}: {len(bad)} labels differ, first at {bad[0].tolist()}")
    assert np.array_equal(got[2], exp[2]), f"{what}: sizes differ"
    assert hk.device_error() == 0
    return got


SHAPES = [(1, 1, 1), (1, 1, 2), (1, 1, 63), (1, 1, 64), (1, 1, 65), (2, 2, 2), (3, 5, 7), (1, 17, 130),
          (33, 1, 1), (17, 33, 65), (16, 16, 64), (5, 40, 129), (20, 3, 200), (2, 70, 2), (31, 31, 31)]


@pytest.mark.parametrize("shape", SHAPES)
def test_shapes_all_masks(hk, shape):
    for p in (0.1, 0.3116, 0.6, 0.95):
        phi = W.percolation(shape, p, seed=hash((shape, p)) % (1 << 30))
        for mask in range(8):
            assert_parity(hk, phi, mask, f"p={p}")


@pytest.mark.parametrize("brick", [(1, 1), (2, 1), (1, 4), (4, 4), (8, 8), (16, 8), (8, 16), (16, 16), (2, 128),
                                   (128, 2), (256, 1), (1, 256), (32, 8)])
def test_brick_shapes(hk, brick):
    hk.set_brick(*brick)
    try:
        rng = np.random.default_rng(brick[0] * 1000 + brick[1])
        for trial in range(6):
            shape = tuple(int(v) for v in rng.integers(1, 90, size=3))
            phi = W.percolation(shape, float(rng.uniform(0.15, 0.7)), seed=trial)
            assert_parity(hk, phi, trial % 8, f"brick={brick}")
        phi = W.percolation((40, 40, 130), 0.3116, seed=5)
        assert_parity(hk, phi, 7, f"brick={brick}")
    finally:
        hk.set_brick(0, 0)


def test_exhaustive_2x2x2(hk):
    for bits in range(256):
        occ = np.array([(bits >> i) & 1 for i in range(8)], dtype=bool).reshape(2, 2, 2)
        phi = np.where(occ, np.float32(1), np.float32(-1))
        for mask in range(8):
            got = gpu_label(hk, phi, mask)
            exp = oracle.label(phi, mask)
            assert got[1] == exp[1] and np.array_equal(got[0], exp[0]) and np.array_equal(got[2], exp[2]), (bits, mask)


def test_adversarial_patterns(hk):
    for shape in [(8, 9, 70), (5, 64, 64), (17, 16, 129)]:
        for mask in (0, 7, 1, 6):
            assert_parity(hk, W.site_checkerboard(shape), mask, "checkerboard")
            assert_parity(hk, W.site_checkerboard(shape, 1), mask, "checkerboard-odd")
            assert_parity(hk, W.constant(shape, 1.0), mask, "full")
            assert_parity(hk, W.constant(shape, -1.0), mask, "empty")
            assert_parity(hk, W.serpentine(shape), mask, "serpentine")
            assert_parity(hk, W.comb(shape), mask, "comb")
    for b in (1, 2, 3, 8):
        assert_parity(hk, W.block_checkerboard((48, 48, 96), (b, b, b)), 7, f"block{b}")


def test_special_values(hk):
    rng = np.random.default_rng(3)
    phi = W.percolation((20, 30, 70), 0.5, seed=9)
    specials = np.array([0x7FC00000, 0x80000000, 0x00000000, 0x00000001, 0x80000001, 0x7F800000, 0xFF800000,
                         0x7F800001, 0x007FFFFF, 0xFFC00000], dtype=np.uint32).view(np.float32)
    idx = rng.integers(0, phi.size, size=5000)
    phi.ravel()[idx] = specials[rng.integers(0, specials.size, size=idx.size)]
    for mask in range(8):
        assert_parity(hk, phi, mask, "specials")


def test_config1(hk):
    phi, mask = W.config(1)
    got = assert_parity(hk, phi, mask, "config1")
    check_invariants(phi, mask, *got)


def test_config4_capsules_full(hk):
    phi, mask = W.config(4)
    got = assert_parity(hk, phi, mask, "config4")
    assert got[1] == 301
    check_invariants(phi, mask, *got, check_connected=False)


def test_config2_droplets_full(hk):
    phi, mask = W.config(2)
    got = assert_parity(hk, phi, mask, "config2")
    check_invariants(phi, mask, *got, check_connected=False)


def test_config3_full(hk):
    """1024^3 periodic at p = 0.3116, the benchmark lattice, in the same
    launch configuration the benchmark times (brick chosen automatically)."""
    phi, mask = W.config(3)
    got = assert_parity(hk, phi, mask, "config3")
    assert 0.045 < got[1] / phi.size < 0.065
    assert int(got[2].sum()) == int((phi > 0).sum())


def test_determinism(hk):
    phi, mask = W.config(1)
    ref = gpu_label(hk, phi, mask)
    for _ in range(20):
        got = gpu_label(hk, phi, mask)
        assert got[1] == ref[1] and np.array_equal(got[0], ref[0]) and np.array_equal(got[2], ref[2])
    phi = W.percolation((256, 256, 256), 0.3116, seed=77)
    ref = assert_parity(hk, phi, 7, "det256")
    for _ in range(5):
        got = gpu_label(hk, phi, 7)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[2], ref[2])


@pytest.mark.parametrize("brick", [(1, 1), (4, 4)])
def test_flatten_race_regression(hk, brick):
    """Node trees must be fully flattened before the final pass: concurrent
    walks once overwrote freshly flattened entries, which showed up as a few
    sites carrying the rank of an intermediate node."""
    shape = (17, 33, 65)
    phi = W.percolation(shape, 0.3116, seed=1234)
    exp = oracle.label(phi, 1)
    hk.set_brick(*brick)
    try:
        for _ in range(30):
            got = gpu_label(hk, phi, 1)
            assert got[1] == exp[1] and np.array_equal(got[0], exp[0]) and np.array_equal(got[2], exp[2])
    finally:
        hk.set_brick(0, 0)
    assert hk.device_error() == 0


def test_no_sizes_and_streams(hk):
    phi_np = W.percolation((30, 40, 100), 0.3116, seed=4)
    phi = torch.from_numpy(phi_np).cuda()
    exp = oracle.label(phi_np, 5)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        lab, k, sz = hk.label(phi, 5, sizes=False)
    s.synchronize()
    assert sz is None and k == exp[1] and np.array_equal(lab.cpu().numpy(), exp[0])


def test_invalid_args_write_nothing(hk):
    import ctypes

    from paper_1405_1931_amd import _lib

    lib = _lib.load()
    phi = torch.ones((4, 4, 4), device="cuda")
    lab = torch.full((4, 4, 4), -7, dtype=torch.int32, device="cuda")
    k = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.hk_label(ctypes.c_void_p(phi.data_ptr()), 4, 4, 4, 9, ctypes.c_void_p(lab.data_ptr()),
                      ctypes.c_void_p(k.data_ptr()), None, st)
    assert rc == _lib.HK_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert (lab == -7).all() and int(k.item()) == -7

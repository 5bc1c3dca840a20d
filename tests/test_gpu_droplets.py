"""GPU parity of the droplet-size statistics (Sec. 5): hk_droplet_stats against
the oracle -- histogram, count and summed size exactly; the sums of R, R^2,
R^3 within rounding.  Each term carries about one ulp from its cube root and
powers, and a sum of K positive terms in any order adds at most K - 1 more
roundings of about one ulp of the total, so 4 K eps relative (eps = 2^-52)
bounds the difference between any two summation orders."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import droplets as D
from paper_1405_1931_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

EPS = 2.0 ** -52


@pytest.fixture(scope="module")
def hk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1405_1931_amd as hk

    hk.set_brick(0, 0)
    return hk


def check(hk, sizes_np, min_size, r_max, n_bins, what):
    print(f"[droplets] {what}: K={sizes_np.size} min {min_size} r_max {r_max} bins {n_bins}", flush=True)
    sizes = torch.from_numpy(np.ascontiguousarray(sizes_np, dtype=np.int64)).cuda()
    if sizes.numel() == 0:
        sizes = torch.zeros(1, dtype=torch.int64, device="cuda")
    k = torch.tensor([sizes_np.size], dtype=torch.int64, device="cuda")
    got = hk.droplet_stats(sizes, k, min_size, r_max, n_bins)
    exp = D.stats(sizes_np, min_size, r_max, n_bins)
    assert np.array_equal(got[0].cpu().numpy(), exp[0]), what
    assert got[1] == exp[1] and got[2] == exp[2], what
    tol = 4.0 * max(1, sizes_np.size) * EPS
    for g, e in zip(got[3:], exp[3:]):
        assert abs(g - e) <= tol * max(1.0, abs(e)), (what, g, e)
    return got


def test_random_sizes(hk):
    rng = np.random.default_rng(11)
    sizes = np.concatenate([rng.integers(1, 40, 20000), rng.integers(40, 2_000_000, 3000), [4188, 4189, 1, 2]])
    for min_size, r_max, n_bins in ((1, 32.0, 64), (3, 12.0, 7), (1, 100.0, 2048), (50, 5.0, 1)):
        check(hk, sizes, min_size, r_max, n_bins, "random sizes")


def test_empty_and_one(hk):
    check(hk, np.zeros(0, dtype=np.int64), 1, 10.0, 8, "no clusters")
    got = check(hk, np.array([1], dtype=np.int64), 1, 1.0, 4, "one site")
    assert got[0].cpu().tolist() == [0, 0, 1, 0]


def test_droplet_field_sizes(hk):
    """Sizes of a labelled droplet field (config 2 at 1/4 and full size)."""
    for scale in (4, 1):
        phi_np, mask = W.config(2, scale)
        phi = torch.from_numpy(phi_np).cuda()
        labels, k, sizes = hk.label(phi, mask)
        s = sizes.cpu().numpy()
        check(hk, s, 1, 40.0, 80, f"droplets 1/{scale}")
        check(hk, s, 27, 40.0, 80, f"droplets 1/{scale}, min 27")
    assert hk.device_error() == 0


def test_argument_errors(hk):
    from paper_1405_1931_amd import _lib

    sizes = torch.ones(4, dtype=torch.int64, device="cuda")
    k = torch.tensor([4], dtype=torch.int64, device="cuda")
    for r_max, n_bins in ((0.0, 4), (-1.0, 4), (float("inf"), 4), (1.0, 0), (1.0, 4096)):
        with pytest.raises(_lib.HkError):
            hk.droplet_stats(sizes, k, 1, r_max, n_bins)


# hk_label_droplets: the statistics gathered by the rank phase itself.  The
# lattices span many rank workgroups (more than the 256 partial
# accumulators at 512^3 and 256^3), partial bricks, no cluster and one.
FUSED_CASES = (
    ("droplets 1/4", lambda: W.config(2, 4)),
    ("droplets full", lambda: W.config(2, 1)),
    ("percolation 256^3 mask 7", lambda: (W.percolation((256, 256, 256), 0.3116, 7), 7)),
    ("percolation 77x45x61 mask 5", lambda: (W.percolation((77, 45, 61), 0.45, 8), 5)),
    ("no occupied site", lambda: (np.full((16, 20, 24), -1.0, dtype=np.float32), 0)),
    ("every site occupied", lambda: (np.ones((16, 20, 24), dtype=np.float32), 7)),
)
FUSED_PARAMS = ((1, 40.0, 80), (27, 12.0, 7), (1, 100.0, 2048), (2, 5.0, 1))


def test_fused_statistics_equal_separate_and_oracle(hk):
    """Labels, K and sizes as hk_label; bins, count and summed size as the
    oracle exactly; the sums of R^k within the summation-order bound."""
    for what, make in FUSED_CASES:
        phi_np, mask = make()
        phi = torch.from_numpy(np.ascontiguousarray(phi_np)).cuda()
        l0, k0, s0 = hk.label(phi, mask)
        s_np = s0.cpu().numpy()
        for min_size, r_max, n_bins in FUSED_PARAMS:
            print(f"[droplets fused] {what}: K={k0} min {min_size} r_max {r_max} bins {n_bins}", flush=True)
            labels, k, sizes, st = hk.label_droplets(phi, mask, min_size, r_max, n_bins)
            assert k == k0 and torch.equal(labels, l0) and torch.equal(sizes, s0), what
            exp = D.stats(s_np, min_size, r_max, n_bins)
            assert np.array_equal(st[0].cpu().numpy(), exp[0]), what
            assert st[1] == exp[1] and st[2] == exp[2], what
            tol = 4.0 * max(1, s_np.size) * EPS
            for g, e in zip(st[3:], exp[3:]):
                assert abs(g - e) <= tol * max(1.0, abs(e)), (what, g, e)
    assert hk.device_error() == 0


def test_fused_statistics_without_sizes_and_repeated(hk):
    """sizes may be NULL; the outputs are written, not accumulated, so two
    calls in a row (into the same tensors, the second on a smaller lattice)
    give the second lattice's statistics alone."""
    dev = "cuda"
    hist = torch.full((80,), 7, dtype=torch.int64, device=dev)
    counts = torch.full((2,), 7, dtype=torch.int64, device=dev)
    sums = torch.full((3,), 7.0, dtype=torch.float64, device=dev)
    for shape, seed in (((96, 80, 72), 3), ((40, 33, 20), 4)):
        print(f"[droplets fused] no sizes: shape {shape}", flush=True)
        phi = torch.from_numpy(W.percolation(shape, 0.3116, seed)).cuda()
        labels = torch.empty_like(phi, dtype=torch.int32)
        k = torch.zeros(1, dtype=torch.int64, device=dev)
        hk.label_droplets_into(phi, 7, labels, k, None, 1, 40.0, 80, hist, counts, sums)
        l0, k0, s0 = hk.label(phi, 7)
        assert int(k.item()) == k0 and torch.equal(labels, l0)
        exp = D.stats(s0.cpu().numpy(), 1, 40.0, 80)
        assert np.array_equal(hist.cpu().numpy(), exp[0])
        assert counts.cpu().tolist() == [exp[1], exp[2]]
        tol = 4.0 * max(1, k0) * EPS
        for g, e in zip(sums.cpu().tolist(), exp[3:]):
            assert abs(g - e) <= tol * max(1.0, abs(e))
    assert hk.device_error() == 0

"""Pins of the droplet-size statistics oracle (Sec. 5: sizes as the radius of
the sphere of equal volume): per-cluster arithmetic with the math module and
the plain floor(R / w) binning, closed forms, filtering and overflow, and
planted mistakes that must fail them."""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import droplets as D


def per_cluster(sizes, min_size, r_max, n_bins):
    """One cluster at a time: R from the volume, bin = floor(R / w), the
    last bin taking everything beyond r_max."""
    w = r_max / n_bins
    hist = [0] * n_bins
    cnt = ssum = 0
    rs = []
    for s in sizes:
        if s < min_size:
            continue
        r = (3.0 * s / (4.0 * math.pi)) ** (1.0 / 3.0)
        hist[min(int(r / w), n_bins - 1)] += 1
        cnt += 1
        ssum += int(s)
        rs.append(r)
    return (np.array(hist), cnt, ssum, math.fsum(rs), math.fsum(r * r for r in rs),
            math.fsum(r ** 3 for r in rs))


def close(a, b, rel=1e-12):
    return abs(a - b) <= rel * max(1.0, abs(a), abs(b))


@pytest.mark.parametrize("seed", range(5))
def test_matches_per_cluster_arithmetic(seed):
    rng = np.random.default_rng(seed)
    sizes = np.concatenate([rng.integers(1, 30, 500), rng.integers(30, 40000, 300), [1, 2, 3, 4188, 4189]])
    for min_size, r_max, n_bins in ((1, 24.0, 24), (5, 30.0, 60), (1, 8.0, 3), (100, 40.0, 1)):
        got = D.stats(sizes, min_size, r_max, n_bins)
        exp = per_cluster(sizes.tolist(), min_size, r_max, n_bins)
        assert np.array_equal(got[0], exp[0]), (seed, min_size, r_max, n_bins)
        assert got[1] == exp[1] and got[2] == exp[2]
        for g, e in zip(got[3:], exp[3:]):
            assert close(g, e, 1e-10), (g, e)


def test_closed_forms():
    # one site: R = (3 / 4 pi)^(1/3)
    h, n, s, r, r2, r3 = D.stats([1], 1, 1.0, 4)
    assert n == 1 and s == 1 and h.tolist() == [0, 0, 1, 0]  # 0.6204 in [0.5, 0.75)
    assert close(r, 0.6203504908994001) and close(r3, 3.0 / (4.0 * math.pi))
    # the sphere of radius 10 holds 4188.79 sites: 4188 falls below R = 10, 4189 above
    h, *_ = D.stats([4188, 4189], 1, 20.0, 20)
    assert h[9] == 1 and h[10] == 1 and h.sum() == 2
    # R^3 sums to 3 S / (4 pi) for any sizes
    sizes = [7, 70, 700, 7000]
    _, _, S, _, _, r3 = D.stats(sizes, 1, 30.0, 10)
    assert S == 7777 and close(r3, 3.0 * 7777 / (4.0 * math.pi))


def test_filter_overflow_and_empty():
    h, n, s, *_ = D.stats([1, 2, 3, 10 ** 9], 3, 10.0, 5)
    assert n == 2 and s == 3 + 10 ** 9
    assert h[-1] == 1  # R = 620 lands in the last bin
    h, n, s, r, r2, r3 = D.stats([], 1, 10.0, 5)
    assert n == 0 and s == 0 and h.sum() == 0 and r == r2 == r3 == 0.0


def _m_square_root(sizes, min_size, r_max, n_bins):
    s = np.asarray(sizes)
    s = s[s >= min_size]
    r = np.sqrt(3.0 * s / (4.0 * math.pi))
    hist = np.bincount(np.minimum((r / (r_max / n_bins)).astype(int), n_bins - 1), minlength=n_bins)
    return (hist, int(s.size), int(s.sum()), math.fsum(r), math.fsum(r * r), math.fsum(r ** 3))


def _m_no_overflow_bin(sizes, min_size, r_max, n_bins):
    out = list(D.stats(sizes, min_size, r_max, n_bins))
    s = np.asarray(sizes)
    s = s[s >= min_size]
    r = np.cbrt(3.0 * s / (4.0 * math.pi))
    out[0] = out[0].copy()
    out[0][-1] -= int((r >= r_max).sum())  # drops the clusters beyond r_max
    return tuple(out)


def _m_ceil_bin(sizes, min_size, r_max, n_bins):
    out = list(D.stats(sizes, min_size, r_max, n_bins))
    s = np.asarray(sizes)
    s = s[s >= min_size]
    r = np.cbrt(3.0 * s / (4.0 * math.pi))
    out[0] = np.bincount(np.minimum(np.ceil(r / (r_max / n_bins)).astype(int), n_bins - 1), minlength=n_bins)
    return tuple(out)


def _m_filter_strict(sizes, min_size, r_max, n_bins):
    return D.stats([s for s in sizes if s > min_size], min_size, r_max, n_bins)


@pytest.mark.parametrize("mutant", [_m_square_root, _m_no_overflow_bin, _m_ceil_bin, _m_filter_strict])
def test_planted_mistakes_fail(mutant):
    rng = np.random.default_rng(3)
    sizes = np.concatenate([rng.integers(1, 50, 300), rng.integers(50, 90000, 200)]).tolist()
    bad = 0
    for min_size, r_max, n_bins in ((1, 24.0, 24), (5, 10.0, 20), (2, 40.0, 7)):
        got = mutant(sizes, min_size, r_max, n_bins)
        exp = per_cluster(sizes, min_size, r_max, n_bins)
        if not (np.array_equal(got[0], exp[0]) and got[1] == exp[1]
                and all(close(g, e, 1e-10) for g, e in zip(got[3:], exp[3:]))):
            bad += 1
    assert bad > 0

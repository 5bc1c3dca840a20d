"""Droplet-size statistics of Sec. 5: TEST INFRASTRUCTURE ONLY.

Same rules as the rest of ``oracle/``: only ``tests/``, ``smoke()`` and
``bench.py``'s cpu_baseline leg may use it; it imports nothing from the
product.

Sec. 5 reports the sizes of the oil domains as the radius of the sphere of
the same volume: a cluster of s sites has R = (3 s / (4 pi))^(1/3) lattice
units.  Written out for the clusters with s >= min_size:

* histogram: n_bins bins of width w = r_max / n_bins over [0, r_max);
  bin i holds the clusters with i w <= R < (i + 1) w, and the last bin also
  takes every R >= r_max.  The bin is decided on the size, without a cube
  root: R >= e  <=>  s >= T(e) = (4 pi / 3) e^3, with the thresholds
  T_i = c * (e_i * e_i * e_i), c = 4.0 * pi / 3.0, e_i = i * w, all in IEEE
  double -- so a bin is an exact integer decision;
* moments: count, sum of s (exact), and sums of R, R^2, R^3 in double
  (R^3 = 3 s / (4 pi); summation order is free, so these carry rounding).
"""
from __future__ import annotations

import math

import numpy as np


def thresholds(r_max, n_bins):
    """T_i for i = 0..n_bins-1, as the definition states them."""
    w = r_max / n_bins
    c = 4.0 * math.pi / 3.0
    out = np.empty(n_bins, dtype=np.float64)
    for i in range(n_bins):
        e = i * w
        out[i] = c * (e * e * e)
    return out


def stats(sizes, min_size, r_max, n_bins):
    """Return (hist int64[n_bins], count, sum_s, sum_r, sum_r2, sum_r3)."""
    s = np.asarray(sizes, dtype=np.int64)
    s = s[s >= min_size]
    T = thresholds(r_max, n_bins)
    # number of thresholds T_1.. T_{n-1} that are <= s
    bins = np.searchsorted(T[1:], s.astype(np.float64), side="right")
    hist = np.bincount(bins, minlength=n_bins).astype(np.int64)
    r = np.cbrt(s.astype(np.float64) * (3.0 / (4.0 * math.pi)))
    return (hist, int(s.size), int(s.sum()), math.fsum(r.tolist()), math.fsum((r * r).tolist()),
            math.fsum((s.astype(np.float64) * (3.0 / (4.0 * math.pi))).tolist()))

"""Pins of the interior/exterior oracle (Sec. 6, last step of the capsule
algorithm): hand-worked fixtures, a plain per-site loop on small random
lattices, the capsule ground truth of the generator, and planted mistakes
that must each fail one of these."""
from __future__ import annotations

import itertools
import os

import numpy as np
import pytest

import oracle
from oracle import classify as C
from paper_1405_1931_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "classify")


def load_fixture(name):
    lines = [ln for ln in open(os.path.join(GOLDEN, name)).read().splitlines()
             if ln.strip() and not ln.startswith("#")]
    it = iter(lines)
    _, nz, ny, nx = next(it).split()
    nz, ny, nx = int(nz), int(ny), int(nx)
    assert next(it).strip() == "I"
    I = np.array([[float(t) for t in next(it).split()] for _ in range(nz * ny)], dtype=np.float32)
    I = I.reshape(nz, ny, nx)
    cases = []
    for ln in it:
        if ln.startswith("mask"):
            case = {"mask": int(ln.split()[1])}
            cases.append(case)
        else:
            key, *vals = ln.split()
            case[key] = [int(v) for v in vals]
    return I, cases


def brute(I, labels, k, mask):
    """The definition, one site and one neighbour at a time."""
    nz, ny, nx = labels.shape
    neg = [0] * k
    pos = [0] * k
    dims = (nx, ny, nz)
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        lab = int(labels[z, y, x])
        if lab <= 0:
            continue
        c = [x, y, z]
        nbrs = set()
        for a in range(3):
            for d in (-1, 1):
                q = list(c)
                q[a] += d
                if mask & (1 << a):
                    q[a] %= dims[a]
                elif not 0 <= q[a] < dims[a]:
                    continue
                if q != c:
                    nbrs.add(tuple(q))
        for qx, qy, qz in nbrs:
            if labels[qz, qy, qx] == 0:
                v = float(I[qz, qy, qx])
                if v < 0:
                    neg[lab - 1] += 1
                elif v > 0:
                    pos[lab - 1] += 1
    inside = [1 if a > b else 0 if b > a else -1 for a, b in zip(neg, pos)]
    return np.array(neg), np.array(pos), np.array(inside)


def cluster_field(I):
    """phi of the HK pass: the sites that kept I0 are the cluster sites."""
    return np.where(I == np.float32(W.I0), np.float32(1), np.float32(-1)).astype(np.float32)


@pytest.mark.parametrize("name", ["plane_ring.txt", "row_ties.txt"])
def test_hand_worked_fixtures(name):
    I, cases = load_fixture(name)
    for case in cases:
        labels, k, _ = oracle.label(cluster_field(I), case["mask"])
        assert k == case["k"][0]
        neg, pos, inside = C.classify(I, labels, k, case["mask"])
        assert neg.tolist() == case["neg"], (name, case["mask"])
        assert pos.tolist() == case["pos"], (name, case["mask"])
        assert inside.tolist() == case["inside"], (name, case["mask"])


def random_case(shape, seed):
    rng = np.random.default_rng(seed)
    I = rng.choice(np.array([W.I0, W.I0, -0.3, -0.01, 0.0, 0.2, 0.45, np.nan], dtype=np.float32),
                   size=shape).astype(np.float32)
    return I


@pytest.mark.parametrize("shape", [(1, 1, 5), (1, 2, 2), (2, 3, 4), (3, 3, 3), (1, 5, 7), (4, 2, 5), (5, 4, 3)])
def test_oracle_equals_per_site_loop(shape):
    for seed in range(6):
        I = random_case(shape, seed + 100 * sum(shape))
        for mask in range(8):
            labels, k, _ = oracle.label(cluster_field(I), mask)
            got = C.classify(I, labels, k, mask)
            exp = brute(I, labels, k, mask)
            for g, e in zip(got, exp):
                assert np.array_equal(g, e), (shape, seed, mask)


def test_capsules_ground_truth():
    """Every capsule interior is inside, the exterior (site 0) outside."""
    shape = (64, 64, 128)
    phi, caps = W.capsules(shape, 10, 6.0, 15.0, 2.0, seed=4)
    I = W.capsule_proximity(shape, caps, 2.0)
    assert np.array_equal(cluster_field(I), phi)
    labels, k, sizes = oracle.label(phi, 4)
    assert k == 11
    neg, pos, inside = C.classify(I, labels, k, 4)
    assert labels.flat[0] == 1
    assert inside[0] == 0 and np.all(inside[1:] == 1)
    # on the lattice a thin stretch of shell can put an inner-half membrane
    # site next to the exterior; the decision is by which side dominates
    assert pos[0] > 10 * neg[0]


def test_empty_and_full():
    I = np.full((3, 4, 5), 0.3, dtype=np.float32)  # no cluster site at all
    labels, k, _ = oracle.label(cluster_field(I), 7)
    assert k == 0
    neg, pos, inside = C.classify(I, labels, k, 7)
    assert neg.size == pos.size == inside.size == 0
    I = np.full((3, 4, 5), W.I0, dtype=np.float32)  # one cluster, no border
    labels, k, _ = oracle.label(cluster_field(I), 7)
    neg, pos, inside = C.classify(I, labels, k, 7)
    assert k == 1 and neg.tolist() == [0] and pos.tolist() == [0] and inside.tolist() == [-1]


# ---------------------------------------------------------------- mutants

def _mutant_no_wrap(I, labels, k, periodic):
    return C.classify(I, labels, k, 0)


def _mutant_sign(I, labels, k, periodic):
    neg, pos, inside = C.classify(I, labels, k, periodic)
    return pos, neg, np.where(pos > neg, 1, np.where(neg > pos, 0, -1)).astype(np.int8)


def _mutant_double_pair(I, labels, k, periodic):
    """counts both neighbours of a periodic length-2 axis"""
    orig = C._neighbour_views

    def views(a, axis, n, per):
        if per and n == 2:
            return [(np.roll(a, 1, axis=axis), None), (np.roll(a, -1, axis=axis), None)]
        return orig(a, axis, n, per)

    C._neighbour_views = views
    try:
        return C.classify(I, labels, k, periodic)
    finally:
        C._neighbour_views = orig


def _mutant_zero_positive(I, labels, k, periodic):
    """counts I == 0 as the positive side"""
    return C.classify(np.where(I == 0, np.float32(0.1), I).astype(np.float32), labels, k, periodic)


@pytest.mark.parametrize("mutant", [_mutant_no_wrap, _mutant_sign, _mutant_double_pair, _mutant_zero_positive])
def test_planted_mistakes_fail_a_pin(mutant):
    failures = 0
    for shape in [(1, 2, 2), (2, 3, 4), (1, 5, 7), (3, 3, 3)]:
        for seed in range(4):
            I = random_case(shape, seed + 7)
            for mask in range(8):
                labels, k, _ = oracle.label(cluster_field(I), mask)
                got = mutant(I, labels, k, mask)
                exp = brute(I, labels, k, mask)
                if not all(np.array_equal(g, e) for g, e in zip(got, exp)):
                    failures += 1
    assert failures > 0

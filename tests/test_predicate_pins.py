"""Pins of the predicate oracle: a table of IEEE single-precision cases
worked out by hand, the same comparisons taken one value at a time in
Python's double arithmetic (exact for float32 values), the labelling of the
occupancy against the brute-force flood fill, and planted mistakes that must
fail these."""
from __future__ import annotations

import struct

import numpy as np
import pytest

from oracle import predicates as P
from pins import bfs_label

F = np.float32
DEN = struct.unpack("<f", struct.pack("<I", 1))[0]  # smallest positive denormal
NAN = float("nan")
INF = float("inf")

# (value, predicate, param, expected occupancy), from the IEEE rules:
# denormals compare by value, +0 == -0, NaN compares false, +-inf are ordered
TABLE = [
    (0.5, "gt", 0.25, True), (0.25, "gt", 0.25, False), (0.0, "gt", -0.0, False), (-0.0, "gt", 0.0, False),
    (DEN, "gt", 0.0, True), (-DEN, "gt", 0.0, False), (DEN, "gt", -DEN, True), (-DEN, "gt", -2 * DEN, True),
    (INF, "gt", 3.0e38, True), (-INF, "gt", -3.0e38, False), (NAN, "gt", -INF, False), (-1.0, "gt", -INF, True),
    (-INF, "gt", -INF, False), (INF, "gt", INF, False),
    (-1.0, "eq", -1.0, True), (-0.0, "eq", 0.0, True), (0.0, "eq", -0.0, True), (NAN, "eq", 0.0, False),
    (DEN, "eq", DEN, True), (DEN, "eq", 0.0, False), (INF, "eq", INF, True), (-1.0000001, "eq", -1.0, False),
]


def py_occupancy(values, predicate, param):
    """One value at a time, in Python floats (float32 -> double is exact)."""
    out = []
    for v in np.asarray(values).ravel().tolist():
        if predicate == "u8":
            out.append(v != 0)
        elif predicate == "gt":
            out.append(v > float(F(param)))
        else:
            out.append(v == float(F(param)))
    return np.array(out, dtype=bool).reshape(np.asarray(values).shape)


def special_field(rng, shape):
    vals = np.array([0.0, -0.0, DEN, -DEN, 1e-38, -1e-38, 0.25, -0.25, 0.5, -1.0, INF, -INF, NAN, 2.0],
                    dtype=np.float32)
    return rng.choice(vals, size=shape).astype(np.float32)


@pytest.mark.parametrize("case", TABLE)
def test_hand_worked_table(case):
    v, pred, t, exp = case
    assert bool(P.occupancy(np.array([v], dtype=np.float32), pred, t)[0]) is exp


def test_equals_scalar_comparisons():
    rng = np.random.default_rng(3)
    # random bit patterns cover NaNs of both signs, denormals and both zeros
    bits = rng.integers(0, 2 ** 32, size=4000, dtype=np.uint64).astype(np.uint32)
    bits[:8] = [0, 0x80000000, 1, 0x80000001, 0x7F800000, 0xFF800000, 0x7FC00000, 0xFFC00001]
    field = bits.view(np.float32)
    for pred, t in (("gt", 0.0), ("gt", -0.0), ("gt", 0.5), ("gt", -2.5e-40), ("eq", 0.0), ("eq", -1.0),
                    ("gt", -INF), ("eq", INF)):
        assert np.array_equal(P.occupancy(field, pred, t), py_occupancy(field, pred, t)), (pred, t)
    bytes_ = rng.integers(0, 256, size=4000).astype(np.uint8)
    assert np.array_equal(P.occupancy(bytes_, "u8"), py_occupancy(bytes_, "u8", 0))


def test_nan_parameter_rejected():
    for pred in ("gt", "eq"):
        with pytest.raises(ValueError):
            P.occupancy(np.zeros(3, np.float32), pred, NAN)


@pytest.mark.parametrize("shape", [(1, 1, 9), (3, 4, 5), (6, 2, 7), (5, 5, 5)])
def test_labels_equal_flood_fill(shape):
    rng = np.random.default_rng(sum(shape))
    field = special_field(rng, shape)
    u8 = rng.integers(0, 3, size=shape).astype(np.uint8) * 127
    for mask in (0, 3, 5, 7):
        for pred, t, f in (("gt", 0.3, field), ("gt", -0.3, field), ("eq", -1.0, field), ("eq", 0.0, field),
                           ("u8", 0, u8)):
            occ = py_occupancy(f, pred, t)
            bl, bk, bs = bfs_label(np.where(occ, F(1), F(-1)).astype(np.float32), mask)
            lab, k, sizes = P.label(f, pred, t, mask)
            assert k == bk and np.array_equal(lab, bl) and np.array_equal(sizes, bs), (pred, t, mask)


def _m_ge(field, predicate, param=0.0):
    if predicate == "gt":
        return np.asarray(field, np.float32) >= np.float32(param)
    return P.occupancy(field, predicate, param)


def _m_bitwise_eq(field, predicate, param=0.0):
    if predicate == "eq":
        return np.asarray(field, np.float32).view(np.uint32) == np.array([param], np.float32).view(np.uint32)[0]
    return P.occupancy(field, predicate, param)


def _m_signed_byte(field, predicate, param=0.0):
    if predicate == "u8":
        return np.asarray(field, np.uint8).view(np.int8) > 0
    return P.occupancy(field, predicate, param)


def _m_nan_equal(field, predicate, param=0.0):
    f = np.asarray(field, np.float32)
    return P.occupancy(field, predicate, param) | (np.isnan(f) if predicate != "u8" else False)


@pytest.mark.parametrize("mutant", [_m_ge, _m_bitwise_eq, _m_signed_byte, _m_nan_equal])
def test_planted_mistakes_fail(mutant):
    bad = 0
    for v, pred, t, exp in TABLE:
        if bool(mutant(np.array([v], np.float32), pred, t)[0]) is not exp:
            bad += 1
    b = np.array([0, 1, 127, 128, 255], dtype=np.uint8)
    if not np.array_equal(mutant(b, "u8"), py_occupancy(b, "u8", 0)):
        bad += 1
    assert bad > 0

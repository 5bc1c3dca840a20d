"""The C-ABI library loads and exports every entry point include/hk.h
declares; host-side argument checks and sizing work without a GPU."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

from paper_1405_1931_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "hk.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(hk_[a-z_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libhk.so not built")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 12
    raw = ctypes.CDLL(_lib.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), f"{n} declared in hk.h but not exported"
    # and the binding knows the signature of each
    assert set(names) <= set(_lib._SIGS)


def test_max_clusters(lib):
    assert lib.hk_max_clusters(1, 1, 1) == 1
    assert lib.hk_max_clusters(3, 5, 7) == 53
    assert lib.hk_max_clusters(1024, 1024, 1024) == 2 ** 29
    assert lib.hk_max_clusters(0, 5, 5) == 0


def test_status_strings(lib):
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert lib.hk_status_string(s).startswith(b"HK_")
    assert b"unknown" in lib.hk_status_string(42)


def test_argument_errors_without_gpu(lib):
    dummy = ctypes.c_void_p(0x1000)
    # null pointers
    assert lib.hk_label(None, 4, 4, 4, 0, dummy, dummy, None, None) == _lib.HK_ERR_INVALID_ARG
    assert lib.hk_label(dummy, 4, 4, 4, 0, None, dummy, None, None) == _lib.HK_ERR_INVALID_ARG
    assert lib.hk_label(dummy, 4, 4, 4, 0, dummy, None, None, None) == _lib.HK_ERR_INVALID_ARG
    # bad edges and masks
    for dims in [(0, 1, 1), (1, -2, 1), (1, 1, 0)]:
        assert lib.hk_label(dummy, *dims, 0, ctypes.c_void_p(0x2000), dummy, None, None) == _lib.HK_ERR_INVALID_ARG
    assert lib.hk_label(dummy, 2, 2, 2, 8, ctypes.c_void_p(0x2000), dummy, None, None) == _lib.HK_ERR_INVALID_ARG
    # labels aliasing phi
    assert lib.hk_label(dummy, 2, 2, 2, 0, dummy, ctypes.c_void_p(0x3000), None, None) == _lib.HK_ERR_INVALID_ARG
    # more than INT32_MAX sites
    assert lib.hk_label(dummy, 2048, 2048, 1024, 0, ctypes.c_void_p(0x2000), dummy, None, None) == _lib.HK_ERR_TOO_LARGE
    # batched: bad count / null table / one bad job rejects the whole call
    assert lib.hk_label_batched(None, 3, None) == _lib.HK_ERR_INVALID_ARG
    assert lib.hk_label_batched(None, -1, None) == _lib.HK_ERR_INVALID_ARG
    assert lib.hk_label_batched(None, 0, None) == _lib.HK_OK
    jobs = (_lib.HkJob * 2)()
    jobs[0] = _lib.HkJob(0x1000, 4, 4, 4, 0, 0x2000, 0x3000, None)
    jobs[1] = _lib.HkJob(0x1000, 4, 0, 4, 0, 0x2000, 0x3000, None)
    assert lib.hk_label_batched(jobs, 2, None) == _lib.HK_ERR_INVALID_ARG


def test_sizing_and_bricks(lib):
    b = lib.hk_workspace_bytes(1024, 1024, 1024)
    assert b > 0
    assert lib.hk_workspace_bytes(0, 1, 1) == _lib.HK_ERR_INVALID_ARG
    by, bz = ctypes.c_int32(), ctypes.c_int32()
    assert lib.hk_get_brick(1024, 1024, 1024, ctypes.byref(by), ctypes.byref(bz)) == 0
    assert by.value * bz.value <= 256 and by.value > 0 and bz.value > 0
    assert lib.hk_set_brick(3, 4) == _lib.HK_ERR_INVALID_ARG
    assert lib.hk_set_brick(32, 16) == _lib.HK_ERR_INVALID_ARG
    assert lib.hk_set_brick(8, 4) == 0
    assert lib.hk_get_brick(100, 100, 100, ctypes.byref(by), ctypes.byref(bz)) == 0
    assert (by.value, bz.value) == (8, 4)
    assert lib.hk_set_brick(0, 0) == 0
    assert lib.hk_set_brick_for_shape(200, 200, 200, 4, 4) == 0
    assert lib.hk_get_brick(220, 250, 130, ctypes.byref(by), ctypes.byref(bz)) == 0
    assert (by.value, bz.value) == (4, 4)
    assert lib.hk_set_brick_for_shape(200, 200, 200, 0, 0) == 0
    jobs = (_lib.HkJob * 3)()
    for i, d in enumerate([(32, 40, 50), (64, 64, 64), (190, 33, 77)]):
        jobs[i] = _lib.HkJob(None, *d, 0, None, None, None)
    assert lib.hk_batched_workspace_bytes(jobs, 3) > 0
    # thin lattices still get a plan
    assert lib.hk_workspace_bytes(1, 1, 1 << 30) > 0
    assert lib.hk_workspace_bytes(1 << 30, 1, 1) > 0


def test_tune_table_save_and_load(lib, tmp_path):
    by, bz = ctypes.c_int32(), ctypes.c_int32()
    assert lib.hk_set_brick_for_shape(300, 90, 70, 8, 16) == 0
    path = str(tmp_path / "bricks.txt").encode()
    assert lib.hk_tune_save(path) == 0
    lines = [l for l in open(path).read().splitlines() if not l.startswith("#")]
    assert "9 7 7 8 16" in lines  # ceil(log2) of 300, 90, 70
    assert lib.hk_set_brick_for_shape(300, 90, 70, 0, 0) == 0
    assert lib.hk_tune_load(path) == 0
    assert lib.hk_get_brick(260, 100, 127, ctypes.byref(by), ctypes.byref(bz)) == 0
    assert (by.value, bz.value) == (8, 16)
    assert lib.hk_set_brick_for_shape(300, 90, 70, 0, 0) == 0
    # malformed files install nothing
    bad = tmp_path / "bad.txt"
    bad.write_text("9 7 7 8 16\n9 7 7 3 16\n")
    assert lib.hk_tune_load(str(bad).encode()) == _lib.HK_ERR_INVALID_ARG
    assert lib.hk_get_brick(300, 90, 70, ctypes.byref(by), ctypes.byref(bz)) == 0
    assert (by.value, bz.value) != (8, 16)
    assert lib.hk_tune_load(str(tmp_path / "missing.txt").encode()) == _lib.HK_ERR_INVALID_ARG
    assert lib.hk_tune_load(None) == _lib.HK_ERR_INVALID_ARG


def test_autotune_argument_errors_without_gpu(lib):
    dummy = ctypes.c_void_p(0x1000)
    by, bz, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float()
    args = (ctypes.byref(by), ctypes.byref(bz), ctypes.byref(ms))
    assert lib.hk_autotune(None, 4, 4, 4, 0, dummy, dummy, None, 3, None, *args) == _lib.HK_ERR_INVALID_ARG
    assert lib.hk_autotune(dummy, 0, 4, 4, 0, dummy, dummy, None, 3, None, *args) == _lib.HK_ERR_INVALID_ARG
    assert lib.hk_autotune(dummy, 4, 4, 4, 9, dummy, dummy, None, 3, None, *args) == _lib.HK_ERR_INVALID_ARG
    assert lib.hk_autotune(dummy, 4, 4, 4, 0, dummy, dummy, None, 0, None, *args) == _lib.HK_ERR_INVALID_ARG
    assert lib.hk_autotune_batched(None, 2, 3, None, *args) == _lib.HK_ERR_INVALID_ARG
    assert lib.hk_autotune_batched(None, 0, 3, None, *args) == _lib.HK_ERR_INVALID_ARG


def test_label_pred_argument_errors_without_gpu(lib):
    dummy = ctypes.c_void_p(0x1000)
    other = ctypes.c_void_p(0x2000)
    nan = float("nan")
    # unknown predicate, NaN threshold or value: rejected before any GPU call
    assert lib.hk_label_pred(dummy, 3, 0.0, 4, 4, 4, 0, other, other, None, None) == _lib.HK_ERR_INVALID_ARG
    assert lib.hk_label_pred(dummy, -1, 0.0, 4, 4, 4, 0, other, other, None, None) == _lib.HK_ERR_INVALID_ARG
    for pred in (_lib.HK_PRED_GT, _lib.HK_PRED_EQ):
        assert lib.hk_label_pred(dummy, pred, nan, 4, 4, 4, 0, other, other, None, None) == _lib.HK_ERR_INVALID_ARG
    # null pointers, bad shapes, labels aliasing the field
    assert lib.hk_label_pred(None, 0, 0.0, 4, 4, 4, 0, other, other, None, None) == _lib.HK_ERR_INVALID_ARG
    assert lib.hk_label_pred(dummy, 2, 0.0, 4, 4, 4, 0, None, other, None, None) == _lib.HK_ERR_INVALID_ARG
    assert lib.hk_label_pred(dummy, 1, 0.0, 0, 4, 4, 0, other, other, None, None) == _lib.HK_ERR_INVALID_ARG
    assert lib.hk_label_pred(dummy, 1, 0.0, 4, 4, 4, 8, other, other, None, None) == _lib.HK_ERR_INVALID_ARG
    assert lib.hk_label_pred(dummy, 0, 0.5, 4, 4, 4, 0, dummy, other, None, None) == _lib.HK_ERR_INVALID_ARG
    assert lib.hk_label_pred(dummy, 0, 0.5, 2048, 2048, 1024, 0, other, other, None, None) == _lib.HK_ERR_TOO_LARGE


def test_label_droplets_argument_errors_without_gpu(lib):
    dummy = ctypes.c_void_p(0x1000)
    o = [ctypes.c_void_p(0x2000 + 0x100 * i) for i in range(6)]
    inf = float("inf")

    def call(phi=dummy, nx=4, mask=0, labels=o[0], k=o[1], r_max=8.0, n_bins=8, hist=o[3], counts=o[4], sums=o[5]):
        return lib.hk_label_droplets(phi, nx, 4, 4, mask, labels, k, o[2], 1, r_max, n_bins, hist, counts, sums, None)

    # the statistics' arguments, as for hk_droplet_stats
    for r_max, n_bins in ((0.0, 8), (-1.0, 8), (inf, 8), (float("nan"), 8), (8.0, 0), (8.0, 2049)):
        assert call(r_max=r_max, n_bins=n_bins) == _lib.HK_ERR_INVALID_ARG
    assert call(hist=None) == _lib.HK_ERR_INVALID_ARG
    assert call(counts=None) == _lib.HK_ERR_INVALID_ARG
    assert call(sums=None) == _lib.HK_ERR_INVALID_ARG
    # the labelling's, as for hk_label
    assert call(phi=None) == _lib.HK_ERR_INVALID_ARG
    assert call(labels=None) == _lib.HK_ERR_INVALID_ARG
    assert call(k=None) == _lib.HK_ERR_INVALID_ARG
    assert call(nx=0) == _lib.HK_ERR_INVALID_ARG
    assert call(mask=8) == _lib.HK_ERR_INVALID_ARG
    assert call(labels=dummy) == _lib.HK_ERR_INVALID_ARG


def test_incremental_argument_errors_without_gpu(lib):
    out = ctypes.c_void_p()
    assert lib.hk_incr_create(0, 4, 4, 0, ctypes.byref(out)) == _lib.HK_ERR_INVALID_ARG
    assert out.value is None
    assert lib.hk_incr_create(4, 4, 4, 9, ctypes.byref(out)) == _lib.HK_ERR_INVALID_ARG
    assert lib.hk_incr_create(2048, 2048, 1024, 0, ctypes.byref(out)) == _lib.HK_ERR_TOO_LARGE
    assert lib.hk_incr_create(4, 4, 4, 0, None) == _lib.HK_ERR_INVALID_ARG
    dummy = ctypes.c_void_p(0x1000)
    assert lib.hk_incr_label(None, dummy, dummy, dummy, None, None, None) == _lib.HK_ERR_INVALID_ARG
    assert lib.hk_incr_device_error(None, None, None) == _lib.HK_ERR_INVALID_ARG
    lib.hk_incr_destroy(None)  # a no-op


def test_int32_site_limit(lib):
    """N <= INT32_MAX: one site more is refused before any device work, the
    largest lattices below it are planned, and thin shapes whose row count
    reaches INT32_MAX are either planned or refused (never an overflow)."""
    dummy = ctypes.c_void_p(0x1000)
    big = (2048, 1024, 1024)  # 2^31 = INT32_MAX + 1 sites
    assert lib.hk_label(dummy, *big, 0, ctypes.c_void_p(0x2000), dummy, None, None) == _lib.HK_ERR_TOO_LARGE
    assert lib.hk_workspace_bytes(*big) == _lib.HK_ERR_TOO_LARGE
    jobs = (_lib.HkJob * 1)()
    jobs[0] = _lib.HkJob(0x1000, *big, 0, 0x2000, 0x3000, None)
    assert lib.hk_label_batched(jobs, 1, None) == _lib.HK_ERR_TOO_LARGE
    assert lib.hk_server_footprint(*big) == _lib.HK_ERR_TOO_LARGE
    # the largest lattice of the GPU tests: 2047 x 1024 x 1024 sites
    n = 2047 * 1024 * 1024
    assert n > 2 ** 30
    assert lib.hk_workspace_bytes(2047, 1024, 1024) > 0
    assert lib.hk_max_clusters(2047, 1024, 1024) == n // 2
    assert lib.hk_max_clusters(2 ** 31 - 1, 1, 1) == 2 ** 30
    for dims in [(1, 2 ** 31 - 1, 1), (1, 1, 2 ** 31 - 1), (2 ** 31 - 1, 1, 1)]:
        v = lib.hk_workspace_bytes(*dims)
        assert v > 0 or v == _lib.HK_ERR_TOO_LARGE, (dims, v)

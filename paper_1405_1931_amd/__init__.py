"""MI355X-native Hoshen-Kopelman cluster labelling (Python binding).

Every step of the labelling runs in the HIP kernels of ``libhk.so``; this
module only checks tensors and passes device pointers and the current HIP
stream through the C-ABI declared in ``include/hk.h``.  PyTorch provides the
device memory and the stream.

    labels, k, sizes = paper_1405_1931_amd.label(phi, periodic=(True, True, True))

``phi`` is a float32 CUDA/HIP tensor of shape (nz, ny, nx); ``labels`` comes
back as int32 of the same shape (0 = medium, clusters 1..K numbered by their
lowest linear site), ``sizes`` as int64[K].
"""
from __future__ import annotations

import ctypes

from . import _lib

__all__ = [
    "label", "label_into", "label_batched", "label_batched_into", "max_clusters", "workspace_bytes",
    "batched_workspace_bytes", "reserve", "release", "set_brick", "get_brick", "set_brick_for_shape",
    "device_error", "mask_of",
]


def mask_of(periodic) -> int:
    if isinstance(periodic, int):
        if not 0 <= periodic <= 7:
            raise ValueError("periodic mask must be in 0..7")
        return periodic
    px, py, pz = periodic
    return (1 if px else 0) | (2 if py else 0) | (4 if pz else 0)


def _stream_handle(stream=None):
    import torch

    if stream is not None:
        return ctypes.c_void_p(stream.cuda_stream)
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if raw is not None:  # the current stream's handle without building a Stream object
        return ctypes.c_void_p(raw(torch.cuda.current_device()))
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_phi(phi):
    import torch

    if not isinstance(phi, torch.Tensor) or phi.dtype != torch.float32 or not phi.is_cuda:
        raise TypeError("phi must be a float32 tensor on the GPU")
    if phi.dim() != 3 or not phi.is_contiguous():
        raise ValueError("phi must be a contiguous (nz, ny, nx) tensor")


def max_clusters(nx: int, ny: int, nz: int) -> int:
    return int(_lib.load().hk_max_clusters(nx, ny, nz))


def workspace_bytes(nx: int, ny: int, nz: int) -> int:
    v = int(_lib.load().hk_workspace_bytes(nx, ny, nz))
    _lib.check(v if v < 0 else 0, "hk_workspace_bytes")
    return v


def label_into(phi, mask, labels, n_clusters, sizes=None, stream=None):
    """Enqueue one labelling into caller-owned tensors; no synchronisation.

    labels: int32 (nz, ny, nx); n_clusters: int64 tensor of >= 1 element;
    sizes: int64 tensor with >= max_clusters entries, or None.
    """
    _check_phi(phi)
    nz, ny, nx = phi.shape
    lib = _lib.load()
    rc = lib.hk_label(
        ctypes.c_void_p(phi.data_ptr()), nx, ny, nz, mask_of(mask),
        ctypes.c_void_p(labels.data_ptr()), ctypes.c_void_p(n_clusters.data_ptr()),
        ctypes.c_void_p(sizes.data_ptr()) if sizes is not None else None,
        _stream_handle(stream),
    )
    _lib.check(rc, "hk_label")


def label(phi, periodic=0, stream=None, sizes=True):
    """Label one lattice; returns (labels int32, K, sizes int64[K] or None).

    Synchronises only to read K back to the host.
    """
    import torch

    _check_phi(phi)
    nz, ny, nx = phi.shape
    labels = torch.empty_like(phi, dtype=torch.int32)
    k = torch.zeros(1, dtype=torch.int64, device=phi.device)
    sz = torch.empty(max(1, max_clusters(nx, ny, nz)), dtype=torch.int64, device=phi.device) if sizes else None
    label_into(phi, periodic, labels, k, sz, stream=stream)
    kk = int(k.item())
    return labels, kk, (sz[:kk] if sz is not None else None)


_PREDICATES = {"gt": _lib.HK_PRED_GT, "eq": _lib.HK_PRED_EQ, "u8": _lib.HK_PRED_U8}


def label_pred_into(field, predicate, param, mask, labels, n_clusters, sizes=None, stream=None):
    """Enqueue the labelling of the sites where `predicate` holds: "gt"
    (field > param), "eq" (field == param) on a float32 field, or "u8"
    (field != 0) on a uint8 field; no synchronisation."""
    import torch

    pk = _PREDICATES[predicate]
    want = torch.uint8 if pk == _lib.HK_PRED_U8 else torch.float32
    if not isinstance(field, torch.Tensor) or field.dtype != want or not field.is_cuda:
        raise TypeError(f"field must be a {want} tensor on the GPU for predicate {predicate!r}")
    if field.dim() != 3 or not field.is_contiguous():
        raise ValueError("field must be a contiguous (nz, ny, nx) tensor")
    nz, ny, nx = field.shape
    rc = _lib.load().hk_label_pred(
        field.data_ptr(), pk, float(param), nx, ny, nz, mask_of(mask), labels.data_ptr(), n_clusters.data_ptr(),
        sizes.data_ptr() if sizes is not None else None, _stream_handle(stream))
    _lib.check(rc, "hk_label_pred")


def label_pred(field, predicate, param=0.0, periodic=0, stream=None):
    """label() for another occupancy predicate (see label_pred_into)."""
    import torch

    nz, ny, nx = field.shape
    labels = torch.empty(field.shape, dtype=torch.int32, device=field.device)
    k = torch.zeros(1, dtype=torch.int64, device=field.device)
    sz = torch.empty(max(1, max_clusters(nx, ny, nz)), dtype=torch.int64, device=field.device)
    label_pred_into(field, predicate, param, periodic, labels, k, sz, stream=stream)
    kk = int(k.item())
    return labels, kk, sz[:kk]


class Incremental:
    """Incremental relabelling state for one lattice shape (hk_incr_*): each
    call labels anew only the bricks whose occupancy changed since the
    previous call, with outputs identical to label()."""

    def __init__(self, shape, periodic=0):
        nz, ny, nx = (int(v) for v in shape)
        h = ctypes.c_void_p()
        _lib.check(_lib.load().hk_incr_create(nx, ny, nz, mask_of(periodic), ctypes.byref(h)), "hk_incr_create")
        self._h = h
        self.shape = (nz, ny, nx)
        self.mask = mask_of(periodic)

    def label_into(self, phi, labels, n_clusters, sizes=None, relabelled=None, stream=None):
        """Enqueue one call; relabelled: int64 device tensor for the number of
        bricks labelled anew, or None."""
        _check_phi(phi)
        if tuple(phi.shape) != self.shape:
            raise ValueError(f"phi has shape {tuple(phi.shape)}, the state was made for {self.shape}")
        if self._h is None:
            raise RuntimeError("the state is closed")
        rc = _lib.load().hk_incr_label(self._h, phi.data_ptr(), labels.data_ptr(), n_clusters.data_ptr(),
                                       sizes.data_ptr() if sizes is not None else None,
                                       relabelled.data_ptr() if relabelled is not None else None,
                                       _stream_handle(stream))
        _lib.check(rc, "hk_incr_label")

    def label(self, phi, stream=None):
        """(labels, K, sizes[K], bricks labelled anew); synchronises for K."""
        import torch

        nz, ny, nx = self.shape
        labels = torch.empty(self.shape, dtype=torch.int32, device=phi.device)
        k = torch.zeros(1, dtype=torch.int64, device=phi.device)
        sz = torch.empty(max(1, max_clusters(nx, ny, nz)), dtype=torch.int64, device=phi.device)
        rel = torch.zeros(1, dtype=torch.int64, device=phi.device)
        self.label_into(phi, labels, k, sz, rel, stream=stream)
        kk = int(k.item())
        return labels, kk, sz[:kk], int(rel.item())

    def device_error(self, stream=None) -> int:
        code = ctypes.c_int32(0)
        _lib.load().hk_incr_device_error(self._h, _stream_handle(stream), ctypes.byref(code))
        return code.value

    def close(self):
        if self._h is not None:
            _lib.load().hk_incr_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _jobs_array(jobs):
    arr = (_lib.HkJob * max(1, len(jobs)))()
    for i, j in enumerate(jobs):
        phi, mask, labels, kbuf, sizes = j
        _check_phi(phi)
        nz, ny, nx = phi.shape
        arr[i] = _lib.HkJob(phi.data_ptr(), nx, ny, nz, mask_of(mask), labels.data_ptr(), kbuf.data_ptr(),
                            sizes.data_ptr() if sizes is not None else None)
    return arr


def batched_workspace_bytes(phis):
    """Workspace bytes of one batched call over tensors (shapes only)."""
    arr = (_lib.HkJob * max(1, len(phis)))()
    for i, phi in enumerate(phis):
        nz, ny, nx = phi.shape
        arr[i] = _lib.HkJob(None, nx, ny, nz, 0, None, None, None)
    v = int(_lib.load().hk_batched_workspace_bytes(arr, len(phis)))
    _lib.check(v if v < 0 else 0, "hk_batched_workspace_bytes")
    return v


def label_batched_into(jobs, stream=None):
    """Enqueue one batched launch.  ``jobs`` is a list of
    (phi, mask, labels, n_clusters, sizes) tensors; no synchronisation."""
    arr = _jobs_array(jobs)
    rc = _lib.load().hk_label_batched(arr, len(jobs), _stream_handle(stream))
    _lib.check(rc, "hk_label_batched")


def label_batched(items, stream=None):
    """Label a list of (phi, periodic) lattices in one batched launch;
    returns a list of (labels, K, sizes[K])."""
    import torch

    jobs = []
    for phi, per in items:
        _check_phi(phi)
        nz, ny, nx = phi.shape
        labels = torch.empty_like(phi, dtype=torch.int32)
        k = torch.zeros(1, dtype=torch.int64, device=phi.device)
        sz = torch.empty(max(1, max_clusters(nx, ny, nz)), dtype=torch.int64, device=phi.device)
        jobs.append((phi, per, labels, k, sz))
    label_batched_into(jobs, stream=stream)
    out = []
    ks = torch.cat([j[3] for j in jobs]).tolist() if jobs else []
    for j, kk in zip(jobs, ks):
        out.append((j[2], int(kk), j[4][: int(kk)]))
    return out


def reserve(nbytes: int, stream=None):
    _lib.check(_lib.load().hk_reserve(int(nbytes), _stream_handle(stream)), "hk_reserve")


def release():
    _lib.load().hk_release()


def set_brick(by: int, bz: int):
    _lib.check(_lib.load().hk_set_brick(by, bz), "hk_set_brick")


def get_brick(nx: int, ny: int, nz: int):
    by, bz = ctypes.c_int32(0), ctypes.c_int32(0)
    _lib.check(_lib.load().hk_get_brick(nx, ny, nz, ctypes.byref(by), ctypes.byref(bz)), "hk_get_brick")
    return by.value, bz.value


def set_brick_for_shape(nx, ny, nz, by, bz):
    _lib.check(_lib.load().hk_set_brick_for_shape(nx, ny, nz, by, bz), "hk_set_brick_for_shape")


def classify_into(I, labels, n_clusters, periodic, neg, pos, inside, stream=None):
    """Enqueue the interior/exterior decision (no synchronisation); output
    tensors hold max_clusters entries."""
    import torch

    _check_phi(I)
    if labels.dtype != torch.int32 or labels.shape != I.shape or not labels.is_contiguous():
        raise ValueError("labels must be a contiguous int32 tensor shaped like I")
    nz, ny, nx = I.shape
    rc = _lib.load().hk_classify(I.data_ptr(), labels.data_ptr(), nx, ny, nz, mask_of(periodic),
                                 n_clusters.data_ptr(), neg.data_ptr(), pos.data_ptr(), inside.data_ptr(),
                                 _stream_handle(stream))
    _lib.check(rc, "hk_classify")


def classify(I, labels, n_clusters, periodic=0, stream=None):
    """(neg, pos, inside)[:K] of every cluster of `labels` (hk_label output on
    the same lattice; n_clusters its device K tensor)."""
    import torch

    nz, ny, nx = I.shape
    cap = max(1, max_clusters(nx, ny, nz))
    neg = torch.empty(cap, dtype=torch.int64, device=I.device)
    pos = torch.empty(cap, dtype=torch.int64, device=I.device)
    inside = torch.empty(cap, dtype=torch.int8, device=I.device)
    classify_into(I, labels, n_clusters, periodic, neg, pos, inside, stream=stream)
    k = int(n_clusters.item())
    return neg[:k], pos[:k], inside[:k]


def droplet_stats_into(sizes, n_clusters, min_size, r_max, n_bins, hist, counts, sums, stream=None):
    """Enqueue the droplet-size statistics of `sizes` (no synchronisation)."""
    rc = _lib.load().hk_droplet_stats(sizes.data_ptr(), n_clusters.data_ptr(), int(sizes.numel()), int(min_size),
                                      float(r_max), int(n_bins), hist.data_ptr(), counts.data_ptr(),
                                      sums.data_ptr(), _stream_handle(stream))
    _lib.check(rc, "hk_droplet_stats")


def droplet_stats(sizes, n_clusters, min_size=1, r_max=32.0, n_bins=64, stream=None):
    """(hist, count, sum of sizes, sum R, sum R^2, sum R^3) of the clusters
    with >= min_size sites, R the radius of the sphere of equal volume."""
    import torch

    dev = sizes.device
    hist = torch.empty(n_bins, dtype=torch.int64, device=dev)
    counts = torch.empty(2, dtype=torch.int64, device=dev)
    sums = torch.empty(3, dtype=torch.float64, device=dev)
    droplet_stats_into(sizes, n_clusters, min_size, r_max, n_bins, hist, counts, sums, stream=stream)
    c = counts.tolist()
    sm = sums.tolist()
    return hist, c[0], c[1], sm[0], sm[1], sm[2]


def label_droplets_into(phi, mask, labels, n_clusters, sizes, min_size, r_max, n_bins, hist, counts, sums,
                        stream=None):
    """Enqueue one labelling with the droplet statistics gathered in the
    pass that finalises the sizes (hk_label_droplets); sizes may be None.
    No synchronisation."""
    _check_phi(phi)
    nz, ny, nx = phi.shape
    rc = _lib.load().hk_label_droplets(
        ctypes.c_void_p(phi.data_ptr()), nx, ny, nz, mask_of(mask),
        ctypes.c_void_p(labels.data_ptr()), ctypes.c_void_p(n_clusters.data_ptr()),
        ctypes.c_void_p(sizes.data_ptr()) if sizes is not None else None,
        int(min_size), float(r_max), int(n_bins),
        ctypes.c_void_p(hist.data_ptr()), ctypes.c_void_p(counts.data_ptr()), ctypes.c_void_p(sums.data_ptr()),
        _stream_handle(stream))
    _lib.check(rc, "hk_label_droplets")


def label_droplets(phi, periodic=0, min_size=1, r_max=32.0, n_bins=64, stream=None):
    """Label one lattice and gather its droplet statistics in the same pass:
    (labels, K, sizes[K], (hist, count, sum of sizes, sum R, sum R^2, sum R^3))."""
    import torch

    _check_phi(phi)
    nz, ny, nx = phi.shape
    dev = phi.device
    labels = torch.empty_like(phi, dtype=torch.int32)
    k = torch.zeros(1, dtype=torch.int64, device=dev)
    sz = torch.empty(max(1, max_clusters(nx, ny, nz)), dtype=torch.int64, device=dev)
    hist = torch.empty(n_bins, dtype=torch.int64, device=dev)
    counts = torch.empty(2, dtype=torch.int64, device=dev)
    sums = torch.empty(3, dtype=torch.float64, device=dev)
    label_droplets_into(phi, periodic, labels, k, sz, min_size, r_max, n_bins, hist, counts, sums, stream=stream)
    kk = int(k.item())
    c = counts.tolist()
    sm = sums.tolist()
    return labels, kk, sz[:kk], (hist, c[0], c[1], sm[0], sm[1], sm[2])


def autotune(phi, periodic=0, reps: int = 3, stream=None):
    """Time every candidate brick shape on this lattice and install the
    fastest for its size bucket; returns (by, bz, ms)."""
    import torch

    _check_phi(phi)
    nz, ny, nx = phi.shape
    labels = torch.empty_like(phi, dtype=torch.int32)
    k = torch.zeros(1, dtype=torch.int64, device=phi.device)
    sz = torch.empty(max(1, max_clusters(nx, ny, nz)), dtype=torch.int64, device=phi.device)
    by, bz, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float()
    rc = _lib.load().hk_autotune(phi.data_ptr(), nx, ny, nz, mask_of(periodic), labels.data_ptr(), k.data_ptr(),
                                 sz.data_ptr(), int(reps), _stream_handle(stream), ctypes.byref(by),
                                 ctypes.byref(bz), ctypes.byref(ms))
    _lib.check(rc, "hk_autotune")
    return by.value, bz.value, ms.value


def autotune_batched(jobs, reps: int = 3, stream=None):
    """One brick shape for the whole batch ``jobs`` (as for label_batched_into),
    installed for every job's size bucket; returns (by, bz, ms)."""
    arr = _jobs_array(jobs)
    by, bz, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float()
    rc = _lib.load().hk_autotune_batched(arr, len(jobs), int(reps), _stream_handle(stream), ctypes.byref(by),
                                         ctypes.byref(bz), ctypes.byref(ms))
    _lib.check(rc, "hk_autotune_batched")
    return by.value, bz.value, ms.value


def tune_save(path: str):
    _lib.check(_lib.load().hk_tune_save(str(path).encode()), "hk_tune_save")


def tune_load(path: str):
    _lib.check(_lib.load().hk_tune_load(str(path).encode()), "hk_tune_load")


def profile_enable(on: bool = True):
    _lib.check(_lib.load().hk_profile_enable(1 if on else 0), "hk_profile_enable")


def profile_read():
    """{kernel name: summed ms} over the hk_label calls profiled since the
    last read, and the number of those calls."""
    lib = _lib.load()
    n = int(lib.hk_phase_count())
    ms = (ctypes.c_float * n)()
    calls = ctypes.c_int32(0)
    _lib.check(lib.hk_profile_read(ms, n, ctypes.byref(calls)), "hk_profile_read")
    return {lib.hk_phase_name(i).decode(): float(ms[i]) for i in range(n)}, calls.value


def device_error(stream=None) -> int:
    code = ctypes.c_int32(0)
    _lib.load().hk_device_error(_stream_handle(stream), ctypes.byref(code))
    return code.value


DEBUG_COUNTERS = ("merge_direct", "roots_direct", "equiv_again", "runs_global")


def debug_counters(stream=None) -> dict:
    """Fallback counters of the workspace of `stream` since the last read
    (hk_debug_counters): how often each bounded fast structure was full."""
    out = (ctypes.c_int64 * len(DEBUG_COUNTERS))()
    _lib.check(_lib.load().hk_debug_counters(_stream_handle(stream), out, len(DEBUG_COUNTERS)),
               "hk_debug_counters")
    return {name: int(out[i]) for i, name in enumerate(DEBUG_COUNTERS)}

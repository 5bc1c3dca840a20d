"""Python handle on the labelling server of libhk.so (argument marshalling only).

The scheduler, admission, batching and latency bookkeeping all run in the
library's native scheduler thread (``hk_server_*`` in include/hk.h); this
module only passes tensors' device pointers in and wraps the arena outputs
as tensors on the way out.
"""
from __future__ import annotations

import ctypes

from . import _check_phi, _lib, _stream_handle, mask_of


class _DeviceArray:
    """A device buffer described by ``__cuda_array_interface__`` (read by
    ``torch.as_tensor``); it does not own the memory."""

    def __init__(self, ptr, shape, typestr):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr, "data": (int(ptr), False),
                                         "version": 3, "strides": None}


class Server:
    """Continuous-batching labelling server on the current device.

    ``arena_bytes`` of device memory are allocated once; each request takes
    ``footprint(shape)`` bytes of it while it runs and keeps its outputs there
    until ``release``.  ``slots`` batches run concurrently, each holding at
    most ``max_batch`` requests.  ``simulate=(fixed_ns, ns_per_site)`` runs the
    same scheduler against a simulated device (no GPU needed; K = 0, no
    outputs)."""

    def __init__(self, arena_bytes: int, slots: int = 2, max_batch: int = 256, simulate=None):
        self._lib = _lib.load()
        h = ctypes.c_void_p()
        if simulate is None:
            rc = self._lib.hk_server_create(int(arena_bytes), int(slots), int(max_batch), ctypes.byref(h))
        else:
            fixed_ns, ns_site = simulate
            rc = self._lib.hk_server_create_simulated(int(arena_bytes), int(slots), int(max_batch), int(fixed_ns),
                                                      float(ns_site), ctypes.byref(h))
        _lib.check(rc, "hk_server_create")
        self._h = h
        self.simulated = simulate is not None
        self._phi = {}     # keeps every request's phi alive until it is released
        self._shape = {}

    # ----------------------------------------------------------------- clock
    def now_ns(self) -> int:
        return int(self._lib.hk_server_now_ns())

    def footprint(self, shape) -> int:
        nz, ny, nx = shape
        v = int(self._lib.hk_server_footprint(nx, ny, nz))
        _lib.check(v if v < 0 else 0, "hk_server_footprint")
        return v

    # -------------------------------------------------------------- requests
    def submit(self, phi, periodic=0, arrival_ns: int = 0, stream=None) -> int:
        """Queue one lattice (float32 cuda tensor (nz, ny, nx), contiguous).

        The batch that reads phi waits on the device for the work enqueued so
        far on `stream` (default: torch's current stream), so phi may still be
        in the making there."""
        _check_phi(phi)
        nz, ny, nx = phi.shape
        t = ctypes.c_uint64()
        rc = self._lib.hk_server_submit_after(self._h, phi.data_ptr(), nx, ny, nz, mask_of(periodic),
                                              int(arrival_ns), _stream_handle(stream), ctypes.byref(t))
        _lib.check(rc, "hk_server_submit")
        self._phi[t.value] = phi
        self._shape[t.value] = (nz, ny, nx)
        return t.value

    def submit_shape(self, shape, periodic=0, arrival_ns: int = 0) -> int:
        """Queue a request by shape only (simulated servers)."""
        from . import mask_of

        nz, ny, nx = shape
        t = ctypes.c_uint64()
        rc = self._lib.hk_server_submit(self._h, None, nx, ny, nz, mask_of(periodic), int(arrival_ns),
                                        ctypes.byref(t))
        _lib.check(rc, "hk_server_submit")
        self._shape[t.value] = (nz, ny, nx)
        return t.value

    def sim_fail(self, ticket: int, status: int):
        """Simulated servers: plant a failure on a waiting request (status
        HK_ERR_DEVICE fails it alone, another negative status its batch)."""
        _lib.check(self._lib.hk_server_sim_fail(self._h, ticket, int(status)), "hk_server_sim_fail")

    def poll(self, ticket: int) -> bool:
        rc = self._lib.hk_server_poll(self._h, ticket)
        if rc < 0:
            _lib.check(rc, "hk_server_poll")
        return rc == 1

    def wait(self, ticket: int, timeout_s: float = 60.0):
        _lib.check(self._lib.hk_server_wait(self._h, ticket, int(timeout_s * 1e9)), "hk_server_wait")

    def drain(self, timeout_s: float = 60.0):
        _lib.check(self._lib.hk_server_drain(self._h, int(timeout_s * 1e9)), "hk_server_drain")

    def result(self, ticket: int, copy: bool = True):
        """(labels (nz, ny, nx) int32, K, sizes[:K] int64, latency_ns) of a done
        request; with copy=False the tensors are views of the arena, valid
        until release(ticket)."""
        import torch

        lab, siz = ctypes.c_void_p(), ctypes.c_void_p()
        k, lat = ctypes.c_int64(), ctypes.c_int64()
        rc = self._lib.hk_server_result(self._h, ticket, ctypes.byref(lab), ctypes.byref(k), ctypes.byref(siz),
                                        ctypes.byref(lat))
        _lib.check(rc, "hk_server_result")
        kk = int(k.value)
        if self.simulated:
            return None, kk, None, int(lat.value)
        shape = self._shape[ticket]
        labels = torch.as_tensor(_DeviceArray(lab.value, shape, "<i4"), device="cuda")
        sizes = torch.as_tensor(_DeviceArray(siz.value, (max(kk, 1),), "<i8"), device="cuda")[:kk]
        if copy:
            labels, sizes = labels.clone(), sizes.clone()
        return labels, kk, sizes, int(lat.value)

    def latency_ns(self, ticket: int) -> int:
        """Latency of a done request (completion observed - arrival)."""
        lat = ctypes.c_int64()
        rc = self._lib.hk_server_result(self._h, ticket, None, None, None, ctypes.byref(lat))
        _lib.check(rc, "hk_server_result")
        return int(lat.value)

    def release(self, ticket: int):
        _lib.check(self._lib.hk_server_release(self._h, ticket), "hk_server_release")
        self._phi.pop(ticket, None)
        self._shape.pop(ticket, None)

    # ------------------------------------------------------------ statistics
    def stats(self) -> dict:
        st = _lib.HkServerStats()
        _lib.check(self._lib.hk_server_read_stats(self._h, ctypes.byref(st)), "hk_server_read_stats")
        return {name: getattr(st, name) for name, _ in _lib.HkServerStats._fields_}

    def reset_stats(self):
        _lib.check(self._lib.hk_server_reset_stats(self._h), "hk_server_reset_stats")

    def close(self):
        if self._h:
            _lib.check(self._lib.hk_server_destroy(self._h), "hk_server_destroy")
            self._h = None
            self._phi.clear()
            self._shape.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

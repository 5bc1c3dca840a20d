"""Serial Hoshen-Kopelman oracle: TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls anything in here, and this
package imports nothing from the product.

``label(phi, periodic)`` runs the plain C implementation in ``hk_oracle.c``
(serial HK rules 1-3 of Sec. 2, label-of-labels list of Sec. 3, periodic wrap
equivalences, compaction to 1..K, sizes by counting as in Sec. 5).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hk_oracle.c")
_LIB = os.path.join(_HERE, "libhk_oracle.so")
_lib = None


def build(src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle with gcc (no fast-math: NaN and denormal compares
    must follow IEEE)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math", "-o", out + ".tmp", src]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _bind(path: str):
    lib = ctypes.CDLL(path)
    lib.hk_oracle_label.argtypes = [
        ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
    ]
    lib.hk_oracle_label.restype = ctypes.c_int
    lib.hk_oracle_max_clusters.argtypes = [ctypes.c_int32] * 3
    lib.hk_oracle_max_clusters.restype = ctypes.c_int64
    return lib


def load(path: str | None = None):
    """Load the compiled oracle, building it first if it is absent."""
    global _lib
    if path is not None:
        return _bind(path)
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _bind(_LIB)
    return _lib


def mask_of(periodic) -> int:
    """(px, py, pz) booleans or an int mask -> bit mask (bit 0 = x)."""
    if isinstance(periodic, (int, np.integer)):
        return int(periodic)
    px, py, pz = periodic
    return (1 if px else 0) | (2 if py else 0) | (4 if pz else 0)


def label(phi: np.ndarray, periodic=0, lib=None):
    """Label a float32 lattice of shape (nz, ny, nx).

    Returns (labels int32 (nz, ny, nx), K, sizes int64[K]).
    """
    lib = lib or load()
    phi = np.ascontiguousarray(phi, dtype=np.float32)
    if phi.ndim != 3:
        raise ValueError("phi must have shape (nz, ny, nx)")
    nz, ny, nx = phi.shape
    labels = np.empty(phi.shape, dtype=np.int32)
    kmax = int(lib.hk_oracle_max_clusters(nx, ny, nz))
    sizes = np.empty(max(kmax, 1), dtype=np.int64)
    k = ctypes.c_int64(0)
    rc = lib.hk_oracle_label(
        phi.ctypes.data, nx, ny, nz, mask_of(periodic),
        labels.ctypes.data, ctypes.addressof(k), sizes.ctypes.data,
    )
    if rc != 0:
        raise RuntimeError(f"hk_oracle_label failed with status {rc}")
    return labels, int(k.value), sizes[: k.value].copy()

"""Occupancy predicates other than phi > 0: TEST INFRASTRUCTURE ONLY.

Same rules as the rest of ``oracle/``: only ``tests/``, ``smoke()`` and
``bench.py``'s cpu_baseline leg may use it; it imports nothing from the
product.

Sec. 2 labels the sites with phi > 0.  The interior detection of Sec. 6
labels the sites whose proximity value I still equals the far-field value
I0, and a caller may also hold another threshold or a ready byte mask.  The
labelling itself is unchanged: the occupancy is computed first, written out
as the plain comparison in IEEE single precision (numpy on float32 values,
which compares denormals by value, +0 equal to -0, and NaN false), and the
serial oracle labels it:

* ``"gt"``: field > param;
* ``"eq"``: field == param;
* ``"u8"``: uint8 field != 0 (param unused).
"""
from __future__ import annotations

import numpy as np

from . import label as _label


def occupancy(field, predicate, param=0.0):
    """Boolean occupancy of `field` under the predicate."""
    if predicate == "u8":
        return np.asarray(field, dtype=np.uint8) != 0
    f = np.asarray(field, dtype=np.float32)
    t = np.float32(param)
    if np.isnan(t):
        raise ValueError("a NaN threshold or value is rejected")
    if predicate == "gt":
        return f > t
    if predicate == "eq":
        return f == t
    raise ValueError(f"unknown predicate {predicate!r}")


def label(field, predicate, param=0.0, periodic=0):
    """(labels, K, sizes) of the sites where the predicate holds."""
    occ = occupancy(field, predicate, param)
    phi = np.where(occ, np.float32(1.0), np.float32(-1.0)).astype(np.float32)
    return _label(phi, periodic)

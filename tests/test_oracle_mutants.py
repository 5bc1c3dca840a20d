"""The pins are strong enough to catch plausible mistakes in the oracle.

Each mutant is a copy of oracle/hk_oracle.c with one plausible slip (a
dropped wrap term, a transposed neighbour, the wrong end of a union, an
off-by-one in compaction, a non-strict occupancy test, ...), compiled into a
temporary library on the CPU.  The pin battery below must pass on the real
oracle and fail on every mutant.  The oracle source itself is never edited.
"""
from __future__ import annotations

import os
import subprocess

import numpy as np
import pytest

import oracle
from golden_io import all_fixtures, load as load_fixture
from paper_1405_1931_amd import workloads as W
from pins import bfs_label

SRC = os.path.join(os.path.dirname(oracle.__file__), "hk_oracle.c")

MUTANTS = {
    "drop_z_wrap": ("if ((mask & 4u) && nz >= 2)", "if (0)"),
    "drop_x_backward": ("if (x > 0 && labels[i - 1] > 0)", "if (0)"),
    "y_for_z_neighbour": ("if (z > 0 && labels[i - sz] > 0)\n                    nb[cnt++] = lol_find(&t, labels[i - sz]);",
                          "if (z > 0 && labels[i - sy] > 0)\n                    nb[cnt++] = lol_find(&t, labels[i - sy]);"),
    "union_keeps_larger": ("if (ra < rb)\n        t->lol[rb] = ra;", "if (ra > rb)\n        t->lol[rb] = ra;"),
    "compaction_off_by_one": ("canon[l] = (int32_t)(++k);", "canon[l] = (int32_t)(k++);"),
    "non_strict_condition": ("!(phi[i] > 0.0f)", "!(phi[i] >= 0.0f)"),
    "wrong_y_wrap_row": ("b = a + sy * (ny - 1);", "b = a + sy * (ny - 1 - (ny > 2));"),
    "rule3_drops_equivalence": ("if (nb[k] != m)\n                            lol_union(&t, m, nb[k]);", "if (nb[k] != m && 0)\n                            lol_union(&t, m, nb[k]);"),
    "sizes_skip_first": ("if (sizes && l > 0)\n            sizes[l - 1] += 1;", "if (sizes && l > 0 && i > 0)\n            sizes[l - 1] += 1;"),
}


def _battery(lib):
    """Return the name of the first failing pin, or None."""
    for name in all_fixtures():
        phi, cases = load_fixture(name)
        for c in cases:
            lab, k, s = oracle.label(phi, c["mask"], lib=lib)
            if k != c["k"] or not np.array_equal(lab, c["labels"]) or not np.array_equal(s, c["sizes"]):
                return f"golden {name} mask {c['mask']}"
    rng = np.random.default_rng(2024)
    for trial in range(40):
        shape = tuple(int(v) for v in rng.integers(1, 9, size=3))
        phi = W.percolation(shape, float(rng.uniform(0.2, 0.8)), seed=trial)
        mask = trial % 8
        lab, k, s = oracle.label(phi, mask, lib=lib)
        lb, kb, sb = bfs_label(phi, mask)
        if k != kb or not np.array_equal(lab, lb) or not np.array_equal(s, sb):
            return f"bfs trial {trial}"
    phi = W.block_checkerboard((16, 16, 16), (2, 2, 2))
    lab, k, s = oracle.label(phi, 7, lib=lib)
    if k != 256:
        return "block checkerboard"
    return None


def _compile(tmp_path, text, tag):
    src = tmp_path / f"{tag}.c"
    src.write_text(text)
    out = tmp_path / f"lib{tag}.so"
    subprocess.run(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-o", str(out), str(src)], check=True)
    return oracle.load(str(out))


def test_battery_passes_on_oracle(tmp_path):
    lib = _compile(tmp_path, open(SRC).read(), "clean")
    assert _battery(lib) is None


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_battery_catches_mutant(mutant, tmp_path):
    old, new = MUTANTS[mutant]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site for {mutant} not found exactly once"
    lib = _compile(tmp_path, text.replace(old, new), mutant)
    assert _battery(lib) is not None, f"mutant {mutant} survived the pins"

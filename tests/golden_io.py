"""Reader for the hand-worked text fixtures in tests/golden/.

Format (lines starting with '#' at column 0 followed by a space are
comments only before 'shape'; lattice rows list x left to right, rows y top
to bottom, planes z separated by blank lines or simply consecutive):

    shape nz ny nx
    phi
    <nz*ny rows; tokens '#' (+1), '.' (-1) or 0xXXXXXXXX float32 bits>
    mask m
    k K
    sizes s1 s2 ...
    labels
    <nz*ny rows of ints>
    (mask/k/sizes/labels blocks repeat)
"""
from __future__ import annotations

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _tok(t):
    if t == "#":
        return np.float32(1.0)
    if t == ".":
        return np.float32(-1.0)
    if t.startswith("0x"):
        return np.array([int(t, 16)], dtype=np.uint32).view(np.float32)[0]
    return np.float32(float(t))


def load(name):
    path = os.path.join(GOLDEN, name)
    with open(path) as f:
        raw = [ln.rstrip("\n") for ln in f]
    lines = []
    started = False
    for ln in raw:
        if not started:
            if ln.startswith("shape"):
                started = True
            else:
                continue
        if ln.startswith("# ") and not ln[2:3] in ("#", ".") and not _looks_like_row(ln):
            continue
        if ln.strip() == "":
            continue
        lines.append(ln)
    it = iter(lines)
    head = next(it).split()
    nz, ny, nx = int(head[1]), int(head[2]), int(head[3])
    assert next(it).strip() == "phi"
    phi = np.empty((nz, ny, nx), dtype=np.float32)
    for r in range(nz * ny):
        toks = next(it).split()
        assert len(toks) == nx, (name, toks)
        phi[r // ny, r % ny, :] = [_tok(t) for t in toks]
    cases = []
    for ln in it:
        if ln.startswith("#"):
            continue
        key, *rest = ln.split()
        if key == "mask":
            cases.append({"mask": int(rest[0])})
        elif key == "k":
            cases[-1]["k"] = int(rest[0])
        elif key == "sizes":
            cases[-1]["sizes"] = np.array([int(v) for v in rest], dtype=np.int64)
        elif key == "labels":
            lab = np.empty((nz, ny, nx), dtype=np.int32)
            for r in range(nz * ny):
                toks = next(it).split()
                lab[r // ny, r % ny, :] = [int(t) for t in toks]
            cases[-1]["labels"] = lab
        else:
            raise ValueError(f"{name}: unexpected line {ln!r}")
    return phi, cases


def _looks_like_row(ln):
    toks = ln.split()
    return all(t in ("#", ".") or t.startswith("0x") for t in toks)


def all_fixtures():
    return sorted(f for f in os.listdir(GOLDEN) if f.endswith(".txt"))

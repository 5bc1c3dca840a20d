"""Seeded synthetic workloads (order-parameter fields ``phi``).

This module only *generates inputs*: it holds none of the labelling
arithmetic (no occupancy test, no neighbour logic, no cluster numbering), so
the oracle side and the GPU side can both consume its arrays.  Every array is
float32 with shape ``(nz, ny, nx)`` (x fastest), produced on the host with
numpy's PCG64 generator from a fixed seed, so both sides see the same bytes.

The paper's own fields come from lattice-Boltzmann runs (Sec. 5 emulsions,
Sec. 6 capsule suspensions) and its benchmark lattice is the block
checkerboard of Sec. 3; none of that data exists here, so these generators
stand in for it:

* ``percolation``   -- i.i.d. site percolation, ``phi = U(0,1) - (1 - p)``.
* ``droplets``      -- emulsion-like field: union of balls, ``tanh`` profile,
                       Gaussian noise (stands in for the Sec. 5 oil droplets).
* ``capsules``      -- closed ellipsoidal shells (``phi = -1``) in a
                       ``phi = +1`` background (stands in for the Sec. 6
                       interior/exterior problem).
* ``block_checkerboard`` -- the Sec. 3 benchmark lattice: rectangular blocks
                       touching only at corners, alternating sign.
* small adversarial patterns (serpentine, comb, site checkerboard, ...).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

F32 = np.float32


def _rng(seed):
    return np.random.default_rng(seed)


# --------------------------------------------------------------------------
# basic fields
# --------------------------------------------------------------------------

def percolation(shape, p, seed, out=None):
    """Site percolation: ``phi = u - (1 - p)`` with ``u ~ U[0,1)`` float32.

    ``shape`` is ``(nz, ny, nx)``.  A site is occupied with probability p.
    """
    rng = _rng(seed)
    if out is None:
        out = rng.random(tuple(shape), dtype=F32)
    else:
        rng.random(out=out, dtype=F32)
    out -= F32(1.0 - p)
    return out


def constant(shape, value):
    return np.full(tuple(shape), F32(value), dtype=F32)


def site_checkerboard(shape, parity=0):
    """+1 where (x + y + z) % 2 == parity, else -1."""
    nz, ny, nx = shape
    z, y, x = np.ogrid[:nz, :ny, :nx]
    return np.where((x + y + z) % 2 == parity, F32(1), F32(-1)).astype(F32)


def block_checkerboard(shape, block):
    """The Sec. 3 benchmark lattice: blocks of ``block = (bz, by, bx)`` sites;
    block (I, J, K) is +1 iff I + J + K is even, else -1.  Equal-sign blocks
    meet only at edges/corners, so each +1 block is its own cluster under
    face connectivity."""
    nz, ny, nx = shape
    bz, by, bx = block
    z, y, x = np.ogrid[:nz, :ny, :nx]
    par = (z // bz + y // by + x // bx) % 2
    return np.where(par == 0, F32(1), F32(-1)).astype(F32)


def serpentine(shape):
    """One long path winding through every other x-row of every other
    z-plane: a single cluster with a maximal-length union chain."""
    nz, ny, nx = shape
    phi = np.full((nz, ny, nx), F32(-1))
    # within each even z-plane: rows y even fully occupied, joined at
    # alternating ends; consecutive even planes joined through odd planes.
    for z in range(0, nz, 2):
        for y in range(0, ny, 2):
            phi[z, y, :] = 1
            if y + 1 < ny and y + 2 < ny:
                end = nx - 1 if (y // 2) % 2 == 0 else 0
                phi[z, y + 1, end] = 1
        if z + 2 < nz:
            last_y = ((ny - 1) // 2) * 2
            end = nx - 1 if (last_y // 2) % 2 == 0 else 0
            phi[z + 1, last_y, end] = 1
    return phi


def comb(shape):
    """A spine along x at y = 0 with teeth along y at every other x,
    repeated on every other z-plane and joined by one column in z."""
    nz, ny, nx = shape
    phi = np.full((nz, ny, nx), F32(-1))
    for z in range(0, nz, 2):
        phi[z, 0, :] = 1
        phi[z, :, ::2] = 1
    if nz > 1:
        phi[:, 0, 0] = 1
    return phi


# --------------------------------------------------------------------------
# emulsion-like droplet field
# --------------------------------------------------------------------------

def _axis_window(c, half, n, periodic):
    """Integer coordinates within ``half`` of centre ``c`` on an axis of
    length n, and their offsets from the centre (minimum image if periodic)."""
    lo = int(math.floor(c - half))
    hi = int(math.ceil(c + half))
    idx = np.arange(lo, hi + 1)
    if periodic:
        if hi - lo + 1 >= n:
            idx = np.arange(n)
            d = idx - c
            d = d - n * np.round(d / n)
            return idx, d
        d = idx - c
        return np.mod(idx, n), d
    keep = (idx >= 0) & (idx < n)
    idx = idx[keep]
    return idx, idx - c


def droplets(shape, n_drops, rmin, rmax, seed, periodic=(True, True, True), noise=0.05,
             width=2.0, margin=8.0):
    """Emulsion-like field: ``n_drops`` balls with radii U[rmin, rmax] and
    uniform random centres; ``sd(x) = max_i (R_i - d_i(x))`` (minimum-image
    distance on periodic axes) evaluated within ``R_i + margin`` of each
    centre; ``phi = tanh(sd / width) + noise * N(0, 1)`` in float32.
    ``periodic`` is (px, py, pz)."""
    nz, ny, nx = shape
    px, py, pz = periodic
    rng = _rng(seed)
    centres = rng.random((n_drops, 3)) * np.array([nx, ny, nz], dtype=np.float64)
    radii = rng.uniform(rmin, rmax, size=n_drops)
    sd = np.full((nz, ny, nx), -np.inf, dtype=F32)
    for (cx, cy, cz), r in zip(centres, radii):
        half = r + margin
        xi, dx = _axis_window(cx, half, nx, px)
        yi, dy = _axis_window(cy, half, ny, py)
        zi, dz = _axis_window(cz, half, nz, pz)
        if xi.size == 0 or yi.size == 0 or zi.size == 0:
            continue
        d = np.sqrt(dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2)
        val = (r - d).astype(F32)
        sub = np.ix_(zi, yi, xi)
        sd[sub] = np.maximum(sd[sub], val)
    phi = np.tanh(sd / F32(width)).astype(F32)
    phi += F32(noise) * rng.standard_normal((nz, ny, nx), dtype=F32)
    return phi


# --------------------------------------------------------------------------
# capsule shells
# --------------------------------------------------------------------------

def _rotation(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


@dataclass
class Capsule:
    centre: np.ndarray       # (cx, cy, cz)
    axes: np.ndarray         # semi-axes (a0, a1, a2)
    rot: np.ndarray          # 3x3, body frame -> lattice frame


def capsules(shape, n_caps, amin, amax, thickness, seed, periodic=(False, False, True),
             gap=2.0, wall=1.0, max_tries=200000):
    """Closed ellipsoidal shells: semi-axes U[amin, amax]^3, uniformly random
    orientation (normalised 4-normal quaternion), centres placed without
    overlap by rejection on bounding spheres (``r = max a`` plus ``gap``) and
    at least ``wall`` sites from non-periodic walls.  Shell sites
    (``f_o <= 1 < f_i`` with ``f_o = sum (u_k / a_k)^2`` and
    ``f_i = sum (u_k / (a_k - thickness))^2`` in the body frame) get
    ``phi = -1``; every other site gets ``+1``.

    Returns (phi, capsules).
    """
    nz, ny, nx = shape
    n_xyz = np.array([nx, ny, nz], dtype=np.float64)
    per = np.array(periodic, dtype=bool)
    rng = _rng(seed)
    caps = []
    tries = 0
    while len(caps) < n_caps:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place capsules without overlap")
        axes = rng.uniform(amin, amax, size=3)
        q = rng.standard_normal(4)
        r = float(axes.max())
        lo = np.where(per, 0.0, r + wall + 1.0)
        hi = np.where(per, n_xyz, n_xyz - r - wall - 2.0)
        if np.any(hi <= lo):
            raise ValueError("lattice too small for capsules")
        c = lo + rng.random(3) * (hi - lo)
        ok = True
        for o in caps:
            d = c - o.centre
            d = np.where(per, d - n_xyz * np.round(d / n_xyz), d)
            if np.linalg.norm(d) < r + float(o.axes.max()) + gap:
                ok = False
                break
        if ok:
            caps.append(Capsule(c, axes, _rotation(q)))
    phi = np.ones((nz, ny, nx), dtype=F32)
    for cap in caps:
        r = float(cap.axes.max()) + 1.0
        xi, dx = _axis_window(cap.centre[0], r, nx, periodic[0])
        yi, dy = _axis_window(cap.centre[1], r, ny, periodic[1])
        zi, dz = _axis_window(cap.centre[2], r, nz, periodic[2])
        fo, fi = _shell_forms(cap, thickness, dx, dy, dz)
        shell = (fo <= 1.0) & (fi > 1.0)
        sub = np.ix_(zi, yi, xi)
        blk = phi[sub]
        blk[shell] = F32(-1)
        phi[sub] = blk
    return phi, caps


def _shell_forms(cap, thickness, dx, dy, dz):
    """Quadratic forms f_o, f_i on the (dz, dy, dx) grid of offsets."""
    D = np.stack(np.broadcast_arrays(dx[None, None, :], dy[None, :, None], dz[:, None, None]), axis=-1)
    u = D @ cap.rot          # lattice offsets -> body frame (rot is orthonormal)
    a = cap.axes
    fo = np.sum((u / a) ** 2, axis=-1)
    fi = np.sum((u / (a - thickness)) ** 2, axis=-1)
    return fo, fi


I0 = -1.0  # proximity value of the sites far from every membrane


def capsule_proximity(shape, caps, thickness, periodic=(False, False, True), i0=I0):
    """Proximity field of the capsule shells, as in the Sec. 6 construction:
    every site far from a membrane keeps ``i0``; a shell site gets a value in
    (-0.5, 0.5) whose sign says on which side of the membrane it lies --
    negative towards the capsule interior, positive towards the outside.
    The membrane is the mid-surface of the shell, ``f_m = 1`` with
    ``f_m = sum (u_k / (a_k - thickness / 2))^2``; the value is
    ``0.05 + 0.4 |tanh(f_m - 1)|`` with the sign of ``f_m - 1`` (never 0).
    The shell sites are exactly the ``phi = -1`` sites of ``capsules``."""
    nz, ny, nx = shape
    out = np.full((nz, ny, nx), F32(i0), dtype=F32)
    for cap in caps:
        r = float(cap.axes.max()) + 1.0
        xi, dx = _axis_window(cap.centre[0], r, nx, periodic[0])
        yi, dy = _axis_window(cap.centre[1], r, ny, periodic[1])
        zi, dz = _axis_window(cap.centre[2], r, nz, periodic[2])
        fo, fi = _shell_forms(cap, thickness, dx, dy, dz)
        shell = (fo <= 1.0) & (fi > 1.0)
        D = np.stack(np.broadcast_arrays(dx[None, None, :], dy[None, :, None], dz[:, None, None]), axis=-1)
        u = D @ cap.rot
        fm = np.sum((u / (cap.axes - thickness / 2.0)) ** 2, axis=-1) - 1.0
        val = (0.05 + 0.4 * np.abs(np.tanh(fm))) * np.where(fm < 0.0, -1.0, 1.0)
        sub = np.ix_(zi, yi, xi)
        blk = out[sub]
        blk[shell] = val[shell].astype(F32)
        out[sub] = blk
    return out


def capsule_interior_counts(shape, caps, thickness, periodic=(False, False, True)):
    """Number of lattice sites with f_i <= 1 for each capsule (the interior
    pocket sizes a correct labelling must report)."""
    nz, ny, nx = shape
    out = []
    for cap in caps:
        r = float(cap.axes.max()) + 1.0
        _, dx = _axis_window(cap.centre[0], r, nx, periodic[0])
        _, dy = _axis_window(cap.centre[1], r, ny, periodic[1])
        _, dz = _axis_window(cap.centre[2], r, nz, periodic[2])
        _, fi = _shell_forms(cap, thickness, dx, dy, dz)
        out.append(int(np.count_nonzero(fi <= 1.0)))
    return out


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------

P_SITE = 0.3116  # site-percolation threshold of the simple cubic lattice

CONFIG_NAMES = {
    1: "percolation 64^3 p=0.3116 non-periodic",
    2: "droplets 512^3 periodic (4000 spheres, R in [6,20])",
    3: "percolation 1024^3 p=0.3116 periodic",
    4: "capsules 256x256x512 z-periodic (300 ellipsoidal shells)",
    5: "stream of 256 uneven lattices (edges log-uniform in [32,192])",
}


def config(cid: int, scale: int = 1):
    """Return ``(phi, mask)`` for configs 1-4; ``scale`` > 1 divides every
    edge (for quick runs of the same recipe)."""
    if cid == 1:
        n = 64 // scale
        return percolation((n, n, n), P_SITE, seed=1), 0
    if cid == 2:
        n = 512 // scale
        drops = max(1, round(4000 / scale ** 3))
        return droplets((n, n, n), drops, 6.0, 20.0, seed=2), 7
    if cid == 3:
        n = 1024 // scale
        return percolation((n, n, n), P_SITE, seed=3), 7
    if cid == 4:
        shape = (512 // scale, 256 // scale, 256 // scale)
        caps = max(1, round(300 / scale ** 3))
        phi, _ = capsules(shape, caps, 6.0, 15.0, 2.0, seed=4)
        return phi, 4
    raise ValueError(f"config {cid} is not a single lattice")


def capsule_config(scale: int = 1):
    """Config 4 with its proximity field: ``(phi, I, mask)``, where phi > 0
    exactly on the sites that kept I0 (the cluster sites of the HK pass) and
    I is signed on the membrane sites (Sec. 6)."""
    shape = (512 // scale, 256 // scale, 256 // scale)
    caps = max(1, round(300 / scale ** 3))
    phi, cl = capsules(shape, caps, 6.0, 15.0, 2.0, seed=4)
    return phi, capsule_proximity(shape, cl, 2.0), 4


@dataclass
class Job:
    phi: np.ndarray
    mask: int
    kind: str
    seed: int


def stream_shapes(n_jobs=256, seed=5, lo=32, hi=192):
    rng = _rng(seed)
    edges = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=(n_jobs, 3)))).astype(int)
    return rng, [(int(e[2]), int(e[1]), int(e[0])) for e in edges]   # (nz, ny, nx)


def stream(n_jobs=256, seed=5, lo=32, hi=192):
    """Config 5 job mix: uneven non-cubic lattices, half percolation with
    p ~ U[0.2, 0.5], half droplet fields at the config-2 density, random
    periodic masks, shuffled order."""
    rng, shapes = stream_shapes(n_jobs, seed, lo, hi)
    jobs = []
    half = n_jobs // 2
    for j, shp in enumerate(shapes):
        mask = int(rng.integers(0, 8))
        jseed = int(rng.integers(0, 2**31 - 1))
        per = (bool(mask & 1), bool(mask & 2), bool(mask & 4))
        if j < half:
            p = float(rng.uniform(0.2, 0.5))
            phi = percolation(shp, p, jseed)
            kind = f"percolation p={p:.3f}"
        else:
            n = shp[0] * shp[1] * shp[2]
            drops = max(1, round(4000 * n / 512 ** 3))
            phi = droplets(shp, drops, 6.0, 20.0, jseed, periodic=per)
            kind = f"droplets n={drops}"
        jobs.append(Job(phi, mask, kind, jseed))
    order = rng.permutation(n_jobs)
    return [jobs[i] for i in order]


def poisson_arrivals(n, rate, seed):
    """Arrival times (seconds from 0) of a Poisson stream with ``rate``/s."""
    rng = _rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))

"""Seeded synthetic inputs for the D3Q19 solver and its checks.

This module holds input generators only -- geometry, initial fields, random
test states -- and none of the lattice Boltzmann arithmetic.  It imports
nothing else from this package, so both the GPU path's tests and the CPU
oracle's tests draw identical inputs from it.

Workload recipes (each seeded, stated in the function):
  * ``taylor_green``     -- 2-D Taylor-Green vortex velocity in x, y.
  * ``channel_flags``    -- solid rows at y = 0 and y = ny - 1.
  * ``sphere_pack``      -- non-overlapping random spheres (periodic box).
  * ``smooth_field``     -- random smooth velocity from the lowest Fourier modes.
  * ``random_offsets``   -- random population offsets for exact permutation tests.
"""
import math

import numpy as np

FLAG_SOLID = 1
FLAG_NOFORCE = 2
FLAG_MOVING = 4

_MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 generator (Steele, Lea & Flood, OOPSLA 2014).

    ``uniform()`` returns the top 53 bits of the next output divided by 2^53,
    a double in [0, 1)."""

    def __init__(self, seed: int):
        self.state = int(seed) & _MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))


def taylor_green(shape, u0=0.01):
    """Velocity [3, nz, ny, nx] of a Taylor-Green vortex with one wavelength
    across the box in x and y, cell indices as coordinates:
    u_x = -u0 cos(kx x) sin(ky y), u_y = u0 sin(kx x) cos(ky y), u_z = 0."""
    nz, ny, nx = shape
    kx, ky = 2 * math.pi / nx, 2 * math.pi / ny
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    u = np.zeros((3, nz, ny, nx))
    u[0] = -u0 * np.cos(kx * x) * np.sin(ky * y)
    u[1] = u0 * np.sin(kx * x) * np.cos(ky * y)
    return u


def channel_flags(shape):
    """Solid walls on the rows y = 0 and y = ny - 1; everything else fluid."""
    nz, ny, nx = shape
    f = np.zeros(shape, dtype=np.uint8)
    f[:, 0, :] = FLAG_SOLID
    f[:, ny - 1, :] = FLAG_SOLID
    return f


def couette_flags(shape):
    """Plane Couette channel: a resting wall on the row y = 0 and a moving
    wall (solid + moving bit) on the row y = ny - 1."""
    nz, ny, nx = shape
    f = np.zeros(shape, dtype=np.uint8)
    f[:, 0, :] = FLAG_SOLID
    f[:, ny - 1, :] = FLAG_SOLID | FLAG_MOVING
    return f


def cavity_flags(shape):
    """Lid-driven cavity: a one-cell solid layer on all six faces of the box,
    the whole top plane z = nz - 1 (edges included) being the moving lid."""
    nz, ny, nx = shape
    f = np.zeros(shape, dtype=np.uint8)
    f[0, :, :] = FLAG_SOLID
    f[:, 0, :] = FLAG_SOLID
    f[:, ny - 1, :] = FLAG_SOLID
    f[:, :, 0] = FLAG_SOLID
    f[:, :, nx - 1] = FLAG_SOLID
    f[nz - 1, :, :] = FLAG_SOLID | FLAG_MOVING
    return f


def sphere_pack(shape, solid_fraction, seed, rmin=4.0, rmax=12.0, max_tries=10_000_000):
    """Random non-overlapping spheres in a periodic box until the solid
    fraction reaches ``solid_fraction``.

    Draw order per attempt (SplitMix64(seed).uniform): r = rmin + (rmax-rmin) u,
    then centre (u nx, u ny, u nz).  An attempt is rejected if its periodic
    minimum-image distance to an accepted centre is below r + r_j.  A cell
    (x, y, z) is solid if its minimum-image distance to the centre is <= r.
    Returns uint8 flags [nz, ny, nx]."""
    nz, ny, nx = shape
    dims = np.array([nx, ny, nz], dtype=np.float64)
    if 2 * rmax + 1 > min(nx, ny, nz):
        raise ValueError("box too small for the sphere radii")
    rng = SplitMix64(seed)
    flags = np.zeros(shape, dtype=np.uint8)
    ncell = nx * ny * nz
    target = solid_fraction * ncell
    cap = 1024
    centres = np.zeros((cap, 3))
    radii = np.zeros(cap)
    ncent = 0
    nsolid = 0
    tries = 0
    while nsolid < target:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("sphere_pack: solid fraction not reached")
        r = rmin + (rmax - rmin) * rng.uniform()
        c = np.array([rng.uniform() * nx, rng.uniform() * ny, rng.uniform() * nz])
        if ncent:
            d = centres[:ncent] - c
            d -= dims * np.round(d / dims)
            if np.any(np.einsum("ij,ij->i", d, d) < (r + radii[:ncent]) ** 2):
                continue
        lo = np.floor(c - r).astype(np.int64)
        hi = np.ceil(c + r).astype(np.int64)
        ax = [np.arange(lo[k], hi[k] + 1) for k in range(3)]
        dx = (ax[0] - c[0])[None, None, :]
        dy = (ax[1] - c[1])[None, :, None]
        dz = (ax[2] - c[2])[:, None, None]
        inside = dx * dx + dy * dy + dz * dz <= r * r
        iz = np.mod(ax[2], nz)
        iy = np.mod(ax[1], ny)
        ix = np.mod(ax[0], nx)
        sub = flags[np.ix_(iz, iy, ix)]
        nsolid += int(np.count_nonzero(inside & (sub == 0)))
        sub[inside] = FLAG_SOLID
        flags[np.ix_(iz, iy, ix)] = sub
        if ncent == cap:
            cap *= 2
            centres = np.resize(centres, (cap, 3))
            radii = np.resize(radii, cap)
        centres[ncent] = c
        radii[ncent] = r
        ncent += 1
    return flags


def smooth_field(n, seed, amplitude=0.02, modes=8):
    """Random smooth velocity [3, n, n, n]: for each component c,
    u_c = sum over a, b, d in [0, modes) (not all zero) of
    A cos(2 pi a x/n + p1) cos(2 pi b y/n + p2) cos(2 pi d z/n + p3),
    with A ~ U(-1, 1) and p1, p2, p3 ~ U(0, 2 pi) drawn from SplitMix64(seed)
    in loop order (c, a, b, d), each term drawing A, p1, p2, p3.  The field is
    then scaled so that max over cells of |u|_2 equals ``amplitude``.
    Coordinates are normalised by n, so a seed defines the same continuous
    field at every resolution."""
    rng = SplitMix64(seed)
    t = np.arange(n, dtype=np.float64) / n
    u = np.zeros((3, n, n, n))
    for comp in range(3):
        # cos(k t + p) = cos(k t) cos p - sin(k t) sin p: sum the separable parts.
        coef = np.zeros((2, 2, 2, modes, modes, modes))
        for a in range(modes):
            for b in range(modes):
                for d in range(modes):
                    if a == 0 and b == 0 and d == 0:
                        continue
                    A = 2.0 * rng.uniform() - 1.0
                    p = [2 * math.pi * rng.uniform() for _ in range(3)]
                    cs = [(math.cos(q), -math.sin(q)) for q in p]
                    for i in range(2):
                        for j in range(2):
                            for k in range(2):
                                coef[i, j, k, a, b, d] = A * cs[0][i] * cs[1][j] * cs[2][k]
        k = 2 * math.pi * np.arange(modes)[:, None] * t[None, :]
        basis = np.stack([np.cos(k), np.sin(k)])  # [2, modes, n]
        field = np.einsum("ijkabd,ian,jbm,kdl->lmn", coef, basis, basis, basis, optimize=True)
        u[comp] = field  # [z, y, x] with x the last axis
    mag = np.sqrt((u * u).sum(axis=0)).max()
    return u * (amplitude / mag)


def random_offsets(shape, seed, scale=1e-2, dtype=np.float64):
    """Random population offsets [19, nz, ny, nx], uniform in [-scale, scale],
    from numpy's PCG64 seeded with ``seed``, rounded to ``dtype``."""
    rng = np.random.default_rng(seed)
    g = rng.uniform(-scale, scale, size=(19,) + tuple(shape))
    return g.astype(dtype)


def random_flags(shape, seed, solid_fraction=0.2, noforce_fraction=0.0):
    """Independent random solid cells (and optional no-force bits on fluid
    cells), from numpy's PCG64 seeded with ``seed``."""
    rng = np.random.default_rng(seed)
    f = (rng.random(shape) < solid_fraction).astype(np.uint8) * FLAG_SOLID
    if noforce_fraction > 0:
        nf = (rng.random(shape) < noforce_fraction) & (f == 0)
        f |= nf.astype(np.uint8) * FLAG_NOFORCE
    return f


def shear_waves(shape, seed, amplitude=0.02):
    """A cheap smooth velocity [3, nz, ny, nx] (float32) for large boxes: each
    component is a sum of two single-wavelength sine waves along the two
    other axes, u_x = A1 sin(2 pi y/ny + p1) + A2 sin(2 pi z/nz + p2) and
    cyclically, with A ~ U(-1, 1) and p ~ U(0, 2 pi) from SplitMix64(seed) in
    the order (x: A1 p1 A2 p2, y: ..., z: ...); scaled to max |u_c| <= amplitude."""
    nz, ny, nx = shape
    rng = SplitMix64(seed)
    axes = {0: nx, 1: ny, 2: nz}
    coords = {0: np.arange(nx, dtype=np.float32)[None, None, :],
              1: np.arange(ny, dtype=np.float32)[None, :, None],
              2: np.arange(nz, dtype=np.float32)[:, None, None]}
    u = np.zeros((3,) + tuple(shape), dtype=np.float32)
    for c in range(3):
        others = [a for a in range(3) if a != c]
        terms = []
        for a in others:
            A = 2.0 * rng.uniform() - 1.0
            p = 2 * math.pi * rng.uniform()
            terms.append((A, np.sin(np.float32(2 * math.pi / axes[a]) * coords[a] + np.float32(p))))
        s = abs(terms[0][0]) + abs(terms[1][0])
        u[c] = (np.float32(amplitude * terms[0][0] / s) * terms[0][1]
                + np.float32(amplitude * terms[1][0] / s) * terms[1][1])
    return u

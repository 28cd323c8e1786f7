"""Failure detection on the GPU: a NaN or an infinity that appears in a fluid
population (corrupted input, a 16-bit overflow) is data, not a wall -- the
neighbour that pulls it collides with it, the corruption spreads, and the
FP64 reduction reports a non-finite mass.  The values are written from the
host as ordinary data; no kernel faults or traps."""
import math

import numpy as np
import pytest
import torch

from paper_1112_0850_amd import _abi as A
from paper_1112_0850_amd import inputs as I
from paper_1112_0850_amd.lbm import LBM
from tests import lattice_ref as R
from tests.gpu_util import f_to_grid, grid_to_f, raw_bits, say

pytestmark = pytest.mark.gpu

STORAGES = ["f32", "f16", "bf16", "f64", "f32x"]
SHAPE = (8, 9, 70)


def _pulled_fluid_slot(flags, seed):
    """(i, z, y, x) of a fluid slot whose puller y + c_i is a fluid cell."""
    e, _, _ = R.e_w_opp()
    rng = np.random.default_rng(seed)
    nz, ny, nx = flags.shape
    while True:
        i = int(rng.integers(1, 19))
        z, y, x = (int(rng.integers(0, n)) for n in flags.shape)
        tz, ty, tx = (z + e[i, 2]) % nz, (y + e[i, 1]) % ny, (x + e[i, 0]) % nx
        if flags[z, y, x] & 1 == 0 and flags[tz, ty, tx] & 1 == 0:
            return i, z, y, x


def _flags(moving):
    fl = I.random_flags(SHAPE, 7, solid_fraction=0.2, noforce_fraction=0.1)
    if moving:
        fl |= I.couette_flags(SHAPE)
    return fl


@pytest.mark.parametrize("bad", [math.nan, math.inf, -math.inf])
@pytest.mark.parametrize("moving", [False, True])
@pytest.mark.parametrize("storage", STORAGES)
def test_non_finite_fluid_value_reaches_the_reduction(storage, moving, bad):
    say("failure detection", storage, "moving walls" if moving else "resting walls", bad)
    flags = _flags(moving)
    wall = (0.03, 0.0, 0.0) if moving else (0.0, 0.0, 0.0)
    rng = np.random.default_rng(4)
    u0 = 0.02 * (rng.random((3,) + SHAPE) - 0.5)
    u0[:, flags & 1 == 1] = 0
    sim = LBM(SHAPE, 0.7, (1e-5, 0, 0), storage, flags=flags, wall_u=wall,
              u0=torch.from_numpy(u0).float(), f16_scale_log2=8 if storage == "f16" else 0)
    sim.step(3)
    assert all(math.isfinite(v) for v in sim.reduce().cpu().tolist())
    g = grid_to_f(sim, offsets=True)
    i, z, y, x = _pulled_fluid_slot(flags, 11)
    g[i, z, y, x] = bad
    f_to_grid(sim, g, offsets=True, flags=flags)
    rest, mov = A.lbm_solid_markers(sim.storage)
    assert raw_bits(sim)[i, z, y, x] not in (rest, mov)
    sim.step(1)
    r = sim.reduce().cpu().tolist()
    say(f"  reduction after one step: {r}")
    assert not math.isfinite(r[0])
    sim.step(2)
    rho, _ = sim.macroscopics(f64=True)
    bad_cells = int((~torch.isfinite(rho)).sum())
    say(f"  non-finite cells after three steps: {bad_cells}")
    assert bad_cells > 19


def test_f16_overflow_is_reported():
    """FP16 with a storage scale too large for the flow (2^24 g overflows
    binary16 once |g| > 65504 / 2^24 = 0.0039, and u_x = 0.08 gives offsets
    of 0.013): the overflowed stores are infinities, which propagate -- also
    past moving walls, whose marker is not an infinity."""
    flags = _flags(True)
    u0 = np.zeros((3,) + SHAPE)
    u0[0] = 0.08
    u0[:, flags & 1 == 1] = 0
    sim = LBM(SHAPE, 0.7, (0, 0, 0), "f16", flags=flags, wall_u=(0.03, 0, 0),
              u0=torch.from_numpy(u0).float(), f16_scale_log2=24)
    sim.step(1)
    r = sim.reduce().cpu().tolist()
    say(f"FP16 overflow (s = 24): reduction {r}")
    assert not math.isfinite(r[0])

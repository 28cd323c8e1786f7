"""Parity of the unpadded grid layout (x_align = 1: x_stride = nx, the
domain sweep's "unpadded" points) against the FP64 oracle in every storage:
bit-exact pure streaming with bounce-back, and the porous update over tens
of steps, at row lengths that are not multiples of the 64-cell wave segment
(so segments straddle row ends and rows start at arbitrary byte offsets)."""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1112_0850_amd import inputs as I
from paper_1112_0850_amd.lbm import LBM
from tests.gpu_util import check_solids, f_to_grid, rel_linf, say

pytestmark = pytest.mark.gpu

STORAGES = ["f32", "f16", "bf16", "f64", "f32x"]
NX = [65, 100, 200]


def _round_to(a, storage):
    dt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16,
          "f64": torch.float64, "f32x": torch.float32}[storage]
    return torch.from_numpy(a).to(dt).to(torch.float64).numpy()


@pytest.mark.parametrize("nx", NX)
@pytest.mark.parametrize("storage", STORAGES)
def test_unpadded_pure_streaming_bit_exact(storage, nx):
    shape = (3, 5, nx)
    say("unpadded pure streaming", storage, shape)
    flags = I.random_flags(shape, 29, solid_fraction=0.25, noforce_fraction=0.2)
    g = _round_to(I.random_offsets(shape, 13), storage)
    g[:, flags & 1 == 1] = 0.0
    sim = LBM(shape, math.inf, (0, 0, 0), storage, flags=flags, x_align=1)
    assert sim.x_stride == nx
    f_to_grid(sim, g, offsets=True, flags=flags)
    for n in (1, 2, 3):
        sim.step(1)
        assert np.array_equal(check_solids(sim, flags), O.stream(g, flags, n=n)), n


@pytest.mark.parametrize("nx", NX)
@pytest.mark.parametrize("storage", STORAGES)
def test_unpadded_porous_parity(storage, nx):
    """Porous box 16 x 12 x nx (10% spheres r 2-4), tau 0.6, a 3-component
    force, from a random velocity, 40 steps; FP32 to 1e-5, FP64 to 1e-12,
    FP32 storage with FP64 arithmetic to 1e-6, 16-bit storage stated."""
    shape = (16, 12, nx)
    say("unpadded porous parity", storage, shape)
    flags = I.sphere_pack(shape, 0.10, seed=nx, rmin=2, rmax=4)
    flags |= I.random_flags(shape, nx, solid_fraction=0.0, noforce_fraction=0.1)
    rng = np.random.default_rng(nx)
    u0 = (0.03 * (rng.random((3,) + shape) - 0.5)).astype(np.float32).astype(np.float64)
    u0[:, flags & 1 == 1] = 0
    F, tau, steps = (2e-5, -1e-5, 5e-6), 0.6, 40
    s = 10 if storage == "f16" else 0
    sim = LBM(shape, tau, F, storage, flags=flags, u0=torch.from_numpy(u0).float(), x_align=1,
              f16_scale_log2=s)
    sim.step(steps)
    f = O.step(O.init(shape, flags, None, u0), tau, F, flags, n=steps)
    check_solids(sim, flags)
    rho, u = sim.macroscopics(f64=True)
    rho_r, u_r = O.macroscopics(f, F, flags)
    fl = (flags & 1) == 0
    e_rho, e_u = rel_linf(rho.cpu().numpy(), rho_r, fl), rel_linf(u.cpu().numpy(), u_r, fl)
    say(f"  rel L-inf rho {e_rho:.2e}  u {e_u:.2e}")
    tol = {"f32": 1e-5, "f64": 1e-12, "f32x": 1e-6, "f16": 2e-2, "bf16": 5e-2}[storage]
    assert e_rho <= tol and e_u <= tol

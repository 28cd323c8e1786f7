"""GPU checks on the benchmark workloads at their stated sizes: the channel
(256 x 128 x 128, walls at y = 0 and 127, g_x = 1e-6, tau = 0.6) against the
analytic start-up series after 5000 steps; the exact discrete steady
Poiseuille profile of BGK + half-way bounce-back + Guo forcing; and the
porous 128^3 crop of the 512^3 geometry against the FP64 oracle in every
storage over 1000 steps (FP32 to 1e-5; the 16-bit errors are stated)."""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1112_0850_amd import inputs as I
from paper_1112_0850_amd.lbm import LBM
from tests.gpu_util import rel_linf, say
from tests.test_oracle_dynamics import _poiseuille_exact

pytestmark = pytest.mark.gpu


def _series(ny, tau, F, t, terms=400):
    """Start-up flow from rest between half-way walls (continuum series on
    top of the lattice steady profile)."""
    H = ny - 2
    nu = (tau - 0.5) / 3
    eta = np.arange(ny) - 0.5
    ref = _poiseuille_exact(ny, tau, F)
    for n in range(1, 2 * terms, 2):
        ref = ref - 4 * F * H * H / (nu * math.pi ** 3 * n ** 3) * np.sin(n * math.pi * eta / H) * \
            math.exp(-n * n * math.pi ** 2 * nu * t / H ** 2)
    return ref


@pytest.mark.parametrize("storage", ["f32", "f32x"])
def test_channel_startup_full_size(storage):
    shape, tau, F, t = (128, 128, 256), 0.6, 1e-6, 5000
    say("channel 256x128x128, 5000 steps vs start-up series", storage)
    flags = I.channel_flags(shape)
    sim = LBM(shape, tau, (F, 0, 0), storage, flags=flags).step(t)
    _, u = sim.macroscopics(f64=True)
    ux = u[0].cpu().numpy()
    prof = ux.mean(axis=(0, 2))
    assert np.abs(ux - prof[None, :, None]).max() <= 1e-6 * prof.max()  # uniform in x, z
    ref = _series(shape[1], tau, F, t)
    err = np.abs(prof[1:-1] - ref[1:-1]).max() / prof.max()
    say(f"  centre u {prof.max():.4e} (F t = {F * t:.1e}); rel deviation from series {err:.2e}")
    assert err <= 0.01
    assert np.abs(u[1:].cpu().numpy()).max() <= 1e-5 * prof.max()  # rounding noise only


# FP32 storage holds the steady state only to ~ulp(|g|)/2 x H^2/(nu pi^2) /
# |u| ~ 1.2e-5 (measured 1.2e-5 with FP32 and 2.5e-5 with FP64 arithmetic):
# the fixed point of the rounded iteration, whatever the arithmetic.
@pytest.mark.parametrize("storage,tol", [("f32", 4e-5), ("f32x", 4e-5), ("f64", 1e-10)])
def test_poiseuille_exact_steady_state_gpu(storage, tol):
    ny, tau, F = 32, 0.6, 1e-6
    shape = (4, ny, 64)
    nu = (tau - 0.5) / 3
    steps = int(1.2 * 12 * (ny - 2) ** 2 / (nu * math.pi ** 2) * math.log(10))
    say("steady Poiseuille", storage, shape, steps, "steps")
    sim = LBM(shape, tau, (F, 0, 0), storage, flags=I.channel_flags(shape)).step(steps)
    _, u = sim.macroscopics(f64=True)
    ux = u[0].cpu().numpy()[:, 1:-1, :]
    ua = _poiseuille_exact(ny, tau, F)[1:-1]
    err = np.abs(ux - ua[None, :, None]).max() / ua.max()
    say(f"  rel error vs exact discrete profile {err:.2e}")
    assert err <= tol


def test_porous_crop_errors_all_storages():
    """128^3 crop of the 512^3 bench geometry, tau = 0.55, g_x = 1e-6, from
    rest, 1000 steps, against the FP64 oracle (errors every 200 steps).
    The stated bar is 1e-5 relative L-inf on rho and u; FP32 is held to 1e-6
    here (observed 2.4e-7 for u at step 1000 with the compensated momentum
    arithmetic, 8.7e-6 without it) and F32X to 1e-6 (observed 7e-8).  FP16
    and BF16 errors are stated, with bounds of about three times the observed
    values as a guard against regressions."""
    steps, chunk, tau, F = 1000, 200, 0.55, (1e-6, 0.0, 0.0)
    flags = np.ascontiguousarray(I.sphere_pack((512, 512, 512), 0.10, seed=12345)[:128, :128, :128])
    shape = flags.shape
    fl = (flags & 1) == 0
    bars = {"f32": 1e-6, "f32x": 1e-6, "f16": 2e-3, "bf16": 2e-2}
    sims = {st: LBM(shape, tau, F, st, flags=flags, f16_scale_log2=s)
            for st, s in (("f32", 0), ("f32x", 0), ("f16", 12), ("bf16", 0))}
    f = O.init(shape, flags)
    m0 = O.reduce(f, F, flags)[0]
    for t in range(chunk, steps + 1, chunk):
        f = O.step(f, tau, F, flags, n=chunk)
        rho_r, u_r = O.macroscopics(f, F, flags)
        say(f"porous 128^3 crop, step {t}: oracle max|u| {np.abs(u_r).max():.3e}")
        for st, sim in sims.items():
            sim.step(chunk)
            rho, u = sim.macroscopics(f64=True)
            rho, u = rho.cpu().numpy(), u.cpu().numpy()
            m = sim.reduce().cpu().numpy()
            e_rho = rel_linf(rho, rho_r, fl)
            e_drho = float(np.abs(rho - rho_r)[fl].max() / np.abs(rho_r - 1)[fl].max())
            e_u = rel_linf(u, u_r, fl)
            say(f"  {st}: rel L-inf rho {e_rho:.2e}  delta-rho {e_drho:.2e}  u {e_u:.2e}  "
                f"mass drift {abs(m[0] - m0) / m0:.2e}")
            assert e_u <= bars[st] and e_rho <= bars[st], (st, t)
"""GPU parity of the two model options against the FP64 oracle: walls moving
with a common velocity (Ladd's corrected half-way bounce-back, reference
density 1; the lid-driven cavity the paper verifies on, Sec. 7) and the
incompressible equilibrium of He & Luo.  Streaming with moving walls, the
cavity and the exact steady plane Couette flow in every storage, the
incompressible Taylor-Green, porous and reduction cases, and the adjoint
kernels and checkpointed rollout gradient with both options."""
import ctypes
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1112_0850_amd import _abi as A
from paper_1112_0850_amd import inputs as I
from paper_1112_0850_amd.lbm import LBM, rollout
from tests.gpu_util import from_nu_grid, to_nu_grid, check_solids, f_to_grid, grid_to_f, rel_linf, say
from tests.test_gpu_forward import _round_to
from tests.test_oracle_adjoint import rollout_grad

pytestmark = pytest.mark.gpu
P = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
STORAGES = ["f32", "f16", "bf16", "f64", "f32x"]


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _moving_flags(shape, seed):
    """Random solids, half of them moving walls, plus no-force cells."""
    fl = I.random_flags(shape, seed, solid_fraction=0.3, noforce_fraction=0.1)
    rng = np.random.default_rng(seed + 1)
    mv = (fl & 1 == 1) & (rng.random(shape) < 0.5)
    return fl | np.where(mv, I.FLAG_MOVING, 0).astype(np.uint8)


@pytest.mark.parametrize("storage", STORAGES)
def test_moving_wall_streaming(storage):
    """tau = +inf, F = 0: pull with bounce-back plus the moving-wall term.
    The GPU adds the rounded term in the storage's arithmetic, so the match
    is to that rounding; the moving-wall cells carry the moving-wall marker."""
    shape = (5, 6, 70)
    uw = (0.04, -0.03, 0.02)
    say("moving-wall streaming", storage, shape)
    flags = _moving_flags(shape, 19)
    g = _round_to(I.random_offsets(shape, 6), storage)
    g[:, flags & 1 == 1] = 0.0
    sim = LBM(shape, math.inf, (0, 0, 0), storage, flags=flags, wall_u=uw)
    f_to_grid(sim, g, offsets=True, flags=flags)
    sim.step(2)
    got = check_solids(sim, flags)
    ref = O.stream(g, flags, n=2, wall_u=uw)
    fl = flags & 1 == 0
    err = np.abs(got - ref)[:, fl].max()
    bound = {"f32": 4e-9, "f32x": 4e-9, "f64": 1e-17, "f16": 6e-5, "bf16": 2e-4}[storage]
    say(f"  max abs error {err:.2e} (bound {bound:.0e})")
    assert err <= bound
    # two steps away from every moving wall the permutation stays exact:
    # random resting solids plus one moving wall row (y = ny - 1)
    fl2 = I.random_flags(shape, 20, solid_fraction=0.25) | I.couette_flags(shape)
    sim2 = LBM(shape, math.inf, (0, 0, 0), storage, flags=fl2, wall_u=uw)
    g2 = g.copy()
    g2[:, fl2 & 1 == 1] = 0.0
    f_to_grid(sim2, g2, offsets=True, flags=fl2)
    sim2.step(2)
    got2 = check_solids(sim2, fl2)
    ref2 = O.stream(g2, fl2, n=2, wall_u=uw)
    far = np.zeros(shape, bool)
    far[:, :shape[1] - 3, :] = True
    assert np.array_equal(got2[:, far], ref2[:, far])
    assert np.abs(got2 - ref2).max() <= bound


CAVITY = (24, 24, 24)
CAVITY_TAU, CAVITY_U = 0.6, 0.05


@pytest.fixture(scope="module")
def cavity_ref():
    fl = I.cavity_flags(CAVITY)
    f = O.step(O.init(CAVITY, fl), CAVITY_TAU, (0, 0, 0), fl, n=300, wall_u=(CAVITY_U, 0, 0))
    return fl, f


@pytest.mark.parametrize("storage,s,tol", [("f32", 0, 1e-5), ("f32x", 0, 1e-6), ("f64", 0, 1e-12),
                                           ("f16", 10, 2e-2), ("bf16", 0, 5e-2)])
def test_lid_driven_cavity_parity(cavity_ref, storage, s, tol):
    """24^3 box, all six faces solid, the top plane moving with (0.05, 0, 0),
    tau = 0.6, 300 steps from rest: rho and u against the oracle (16-bit
    storage: the error is stated, with a loose bound), FP64 mass drift."""
    fl, f = cavity_ref
    say("lid-driven cavity", storage, CAVITY)
    sim = LBM(CAVITY, CAVITY_TAU, (0, 0, 0), storage, flags=fl, wall_u=(CAVITY_U, 0, 0),
              f16_scale_log2=s)
    m0 = float(sim.reduce()[0])
    sim.step(300)
    check_solids(sim, fl)
    rho, u = sim.macroscopics(f64=True)
    rho_r, u_r = O.macroscopics(f, (0, 0, 0), fl)
    mask = fl & 1 == 0
    e_rho = rel_linf(rho.cpu().numpy(), rho_r, mask)
    e_u = rel_linf(u.cpu().numpy(), u_r, mask)
    drift = abs(float(sim.reduce()[0]) - m0) / m0
    say(f"  rho {e_rho:.2e}  u {e_u:.2e}  mass drift {drift:.1e}")
    assert e_u <= tol and e_rho <= tol
    # FP32 storage rounds every population each step: mass drifts at ~1e-10
    assert drift <= {"f64": 1e-13, "f32": 1e-8, "f32x": 1e-8}.get(storage, 1e-5)


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32x", 2e-5), ("f32", 2e-5)])
def test_couette_exact_steady_state(storage, tol):
    """Plane Couette flow, resting wall y = 0, wall y = ny - 1 moving with
    (U, 0, 0): the steady profile is exactly u_x = U (y - 1/2)/H, H = ny - 2.
    FP32 storage holds a steady state only to about ulp(|g|)/2 x H^2/(nu
    pi^2) / |u|, whatever the arithmetic: FP32 and F32X share that bound."""
    shape, U, tau = (4, 34, 64), 0.05, 1.0
    say("Couette steady state", storage, shape)
    fl = I.couette_flags(shape)
    H, nu = shape[1] - 2, (tau - 0.5) / 3
    steps = int(30 * H * H / (nu * math.pi ** 2))
    sim = LBM(shape, tau, (0, 0, 0), storage, flags=fl, wall_u=(U, 0, 0)).step(steps)
    rho, u = sim.macroscopics(f64=True)
    u = u.cpu().numpy()
    y = np.arange(1, shape[1] - 1)
    ex = (U * (y - 0.5) / H)[None, :, None]
    e = np.abs(u[0][:, 1:-1, :] - ex).max() / U
    say(f"  u_x error {e:.2e} of U (bound {tol:.0e}), {steps} steps")
    assert e <= tol
    assert np.abs(u[1:, :, 1:-1, :]).max() <= tol * U
    assert np.abs(rho.cpu().numpy()[:, 1:-1, :] - 1).max() <= tol


# -- incompressible equilibrium ----------------------------------------------

@pytest.mark.parametrize("storage,tol", [("f32", 1e-5), ("f64", 1e-12), ("f32x", 1e-6)])
def test_incompressible_taylor_green_parity(storage, tol):
    shape, tau = (32, 32, 32), 0.8
    say("incompressible TGV", storage)
    u0 = _f32(I.taylor_green(shape, 0.01))
    sim = LBM(shape, tau, (0, 0, 0), storage, u0=torch.from_numpy(u0).float(),
              equilibrium="incompressible").step(200)
    f = O.step(O.init(shape, None, None, u0, incompressible=True), tau, n=200, incompressible=True)
    rho, u = sim.macroscopics(f64=True)
    rho_r, u_r = O.macroscopics(f, incompressible=True)
    e_rho, e_u = rel_linf(rho.cpu().numpy(), rho_r), rel_linf(u.cpu().numpy(), u_r)
    say(f"  rho {e_rho:.2e}  u {e_u:.2e}")
    assert e_rho <= tol and e_u <= tol


@pytest.mark.parametrize("storage,s,tol", [("f32", 0, 1e-5), ("f64", 0, 1e-12), ("f32x", 0, 1e-6),
                                           ("f16", 12, 2e-2), ("bf16", 0, 5e-2)])
def test_incompressible_porous_moving_walls_parity(storage, s, tol):
    """Random solids (half of them moving walls), no-force cells, body force,
    a ragged 70-cell row and the incompressible equilibrium, 60 steps; the
    FP64 reductions against the oracle's."""
    shape, tau, F, uw = (12, 10, 70), 0.7, (2e-4, -1e-4, 5e-5), (0.03, 0.0, -0.02)
    say("incompressible porous + moving walls", storage, shape)
    flags = _moving_flags(shape, 31)
    rng = np.random.default_rng(3)
    u0 = _f32(0.04 * (rng.random((3,) + shape) - 0.5))
    u0[:, flags & 1 == 1] = 0
    sim = LBM(shape, tau, F, storage, flags=flags, u0=torch.from_numpy(u0).float(), wall_u=uw,
              equilibrium="incompressible", f16_scale_log2=s).step(60)
    f = O.step(O.init(shape, flags, None, u0, incompressible=True), tau, F, flags, n=60, wall_u=uw,
               incompressible=True)
    check_solids(sim, flags)
    rho, u = sim.macroscopics(f64=True)
    rho_r, u_r = O.macroscopics(f, F, flags, incompressible=True)
    m = flags & 1 == 0
    e_rho, e_u = rel_linf(rho.cpu().numpy(), rho_r, m), rel_linf(u.cpu().numpy(), u_r, m)
    r, r_ref = sim.reduce().cpu().numpy(), O.reduce(f, F, flags, incompressible=True)
    e_red = np.abs(r - r_ref) / np.maximum(np.abs(r_ref), 1e-30)
    say(f"  rho {e_rho:.2e}  u {e_u:.2e}  reductions {e_red.max():.2e}")
    assert e_rho <= tol and e_u <= tol
    assert e_red[0] <= tol and e_red[4] <= 10 * tol


# -- adjoint with both options ------------------------------------------------

@pytest.mark.parametrize("inc", [False, True])
def test_adjoint_kernels_vs_oracle(inc):
    """Seed, step and init kernels (pull form: nu = dL/df is carried) with
    moving walls and the chosen equilibrium against the oracle's transposed
    streaming and transposed collision."""
    shape, tau, F, uw = (9, 10, 70), 0.62, (3e-4, -2e-4, 1e-4), (0.04, 0.0, 0.01)
    say("adjoint kernels, moving walls, incompressible =", inc)
    flags = _moving_flags(shape, 55)
    rng = np.random.default_rng(4)
    u0 = _f32(0.03 * (rng.random((3,) + shape) - 0.5))
    u0[:, flags & 1 == 1] = 0
    fn = O.step(O.init(shape, flags, None, u0, incompressible=inc), tau, F, flags, n=3, wall_u=uw,
                incompressible=inc)
    nu1 = _f32(rng.standard_normal((19,) + shape))
    nu1[:, flags & 1 == 1] = 0
    eq = "incompressible" if inc else "qian"
    sim = LBM(shape, tau, F, "f32", flags=flags, wall_u=uw, equilibrium=eq)
    f_to_grid(sim, fn, flags=flags)
    fprev = grid_to_f(sim)
    f_pre = O.stream(fprev, flags, wall_u=uw)
    # step
    nt1 = to_nu_grid(sim, nu1, flags)
    nt0 = torch.zeros_like(nt1)
    part = torch.zeros(sim.adj_partials_bytes // 8, dtype=torch.float64, device="cuda")
    A.lbm_adjoint_step(sim.ctx, P(sim.grids[sim.current]), P(nt1), P(nt0), P(part))
    dF = torch.empty(3, dtype=torch.float64, device="cuda")
    A.lbm_adjoint_finish_dF(sim.ctx, P(part), P(dF))
    torch.cuda.synchronize()
    ref, dF_ref = O.adjoint_collide(f_pre, O.stream_transpose(nu1, flags), tau, F, flags,
                                    incompressible=inc)
    e, eF = rel_linf(from_nu_grid(sim, nt0, flags), ref), np.abs(dF.cpu().numpy() - dF_ref).max() / \
        np.abs(dF_ref).max()
    say(f"  step: nu {e:.2e}, dL/dF {eF:.2e}")
    assert e <= 1e-5 and eF <= 1e-5
    # seed
    gr, gu = _f32(rng.standard_normal(shape)), _f32(rng.standard_normal((3,) + shape))
    grt, gut = torch.from_numpy(gr).float().cuda(), torch.from_numpy(gu).float().cuda()
    nu = torch.zeros(sim.grid_bytes // 4, dtype=torch.float32, device="cuda")
    A.lbm_adjoint_seed(sim.ctx, P(sim.grids[sim.current]), P(grt), P(gut), P(nu), P(part))
    A.lbm_adjoint_finish_dF(sim.ctx, P(part), P(dF))
    fT = O.step(fprev, tau, F, flags, wall_u=uw, incompressible=inc)
    lam_ref, dF1 = O.adjoint_seed(fT, gr, gu, F, flags, incompressible=inc)
    nu_ref, dF2 = O.adjoint_collide(f_pre, lam_ref, tau, F, flags, incompressible=inc)
    torch.cuda.synchronize()
    e, eF = rel_linf(from_nu_grid(sim, nu, flags), nu_ref), \
        np.abs(dF.cpu().numpy() - (dF1 + dF2)).max() / np.abs(dF1 + dF2).max()
    say(f"  seed: nu {e:.2e}, dL/dF {eF:.2e}")
    assert e <= 1e-5 and eF <= 1e-5
    # init, with a non-uniform rho0
    rho0 = _f32(1 + 0.02 * (rng.random(shape) - 0.5))
    du0 = torch.empty((3,) + shape, dtype=torch.float32, device="cuda")
    rho0t, u0t = torch.from_numpy(rho0).float().cuda(), torch.from_numpy(u0).float().cuda()
    A.lbm_adjoint_init(sim.ctx, P(nt1), P(rho0t), P(u0t), P(du0))
    ref, _ = O.adjoint_init(O.stream_transpose(nu1, flags), u0, flags, rho0=rho0,
                            incompressible=inc)
    torch.cuda.synchronize()
    assert rel_linf(du0.double().cpu().numpy(), ref) <= 1e-6


@pytest.mark.parametrize("inc", [False, True])
def test_cavity_rollout_gradient_vs_oracle(inc):
    """16^3 lid-driven box with random obstacles, 30 steps, checkpoints every
    7: the rollout's gradients against the oracle's reverse sweep."""
    n, tau, steps, uw = 16, 0.6, 30, (0.03, 0.0, 0.01)
    shape = (n, n, n)
    say("cavity rollout gradient vs oracle adjoint, incompressible =", inc)
    flags = I.random_flags(shape, 13, solid_fraction=0.05, noforce_fraction=0.1) | \
        I.cavity_flags(shape)
    u0 = _f32(I.smooth_field(n, 2024, amplitude=0.02, modes=4))
    u0[:, flags & 1 == 1] = 0
    target = _f32(I.smooth_field(n, 7, amplitude=0.02, modes=4))
    F = np.array([1e-4, -5e-5, 2e-5])
    u0t = torch.from_numpy(u0).float().cuda().requires_grad_(True)
    g = torch.tensor(F, dtype=torch.float64, requires_grad=True)
    eq = "incompressible" if inc else "qian"
    rho, u = rollout(u0t, g, steps=steps, tau=tau, flags=flags, checkpoint_every=7, wall_u=uw,
                     equilibrium=eq)
    fl = torch.from_numpy((flags & 1) == 0).cuda()
    loss = ((u - torch.from_numpy(target).float().cuda()) ** 2)[:, fl].mean()
    loss.backward()
    du0_ref, dF_ref = rollout_grad(u0, F, flags, tau, steps, target, uw, inc)
    e_u = rel_linf(u0t.grad.double().cpu().numpy(), du0_ref)
    e_F = np.abs(g.grad.numpy() - dF_ref).max() / np.abs(dF_ref).max()
    say(f"  dL/du0 {e_u:.2e}, dL/dg {e_F:.2e}")
    assert e_u <= 1e-4 and e_F <= 1e-4


# -- the split design: a separate obstacle kernel ------------------------------

@pytest.mark.parametrize("storage", STORAGES)
def test_separate_obstacle_kernel(storage):
    """obstacle_kernel = 1 (the paper's split design, Sec. 7): with resting
    and moving walls, body force and no-force cells, FP32 and FP64 storage
    give the fused design's states bit for bit (both round the bounced value
    once, in the storage precision); every storage matches the oracle."""
    shape, tau, F, uw = (12, 10, 70), 0.7, (2e-4, -1e-4, 5e-5), (0.03, 0.0, -0.02)
    say("separate obstacle kernel", storage, shape)
    flags = _moving_flags(shape, 47)
    rng = np.random.default_rng(9)
    u0 = _f32(0.04 * (rng.random((3,) + shape) - 0.5))
    u0[:, flags & 1 == 1] = 0
    s = 12 if storage == "f16" else 0
    kw = dict(flags=flags, u0=torch.from_numpy(u0).float(), wall_u=uw, f16_scale_log2=s)
    split = LBM(shape, tau, F, storage, obstacle_kernel=1, **kw).step(50)
    check_solids(split, flags)
    if storage in ("f32", "f64"):
        fused = LBM(shape, tau, F, storage, **kw).step(50)
        # raw bytes: the solid cells' NaN markers compare equal this way
        assert torch.equal(split.grids[split.current], fused.grids[fused.current])
    f = O.step(O.init(shape, flags, None, u0), tau, F, flags, n=50, wall_u=uw)
    rho, u = split.macroscopics(f64=True)
    rho_r, u_r = O.macroscopics(f, F, flags)
    m = flags & 1 == 0
    e_u = rel_linf(u.cpu().numpy(), u_r, m)
    say(f"  u vs oracle {e_u:.2e}")
    assert e_u <= {"f32": 1e-5, "f64": 1e-12, "f32x": 1e-6, "f16": 2e-2, "bf16": 5e-2}[storage]

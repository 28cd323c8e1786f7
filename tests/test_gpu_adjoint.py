"""GPU parity of the discrete adjoint: each adjoint kernel against the FP64
oracle's adjoint, the full checkpointed rollout gradient against the
oracle's reverse sweep and against FP64 central finite differences of the
oracle's forward map, and bit-identical gradients for any checkpoint spacing."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1112_0850_amd import _abi as A
from paper_1112_0850_amd import inputs as I
from paper_1112_0850_amd.lbm import LBM, rollout
from tests.gpu_util import f_to_grid, from_nu_grid, grid_to_f, rel_linf, say, to_nu_grid
from tests.test_oracle_adjoint import rollout_grad, rollout_loss

pytestmark = pytest.mark.gpu
P = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def case():
    shape = (9, 10, 70)
    flags = I.random_flags(shape, 77, solid_fraction=0.2, noforce_fraction=0.15)
    rng = np.random.default_rng(4)
    u0 = 0.03 * (rng.random((3,) + shape) - 0.5)
    u0[:, flags & 1 == 1] = 0
    tau, F = 0.62, (3e-4, -2e-4, 1e-4)
    fn = O.step(O.init(shape, flags, None, _f32(u0)), tau, F, flags, n=3)
    nu1 = rng.standard_normal((19,) + shape)
    nu1[:, flags & 1 == 1] = 0
    return dict(shape=shape, flags=flags, tau=tau, F=F, fn=fn, nu1=_f32(nu1), u0=_f32(u0))


def _sim(c):
    return LBM(c["shape"], c["tau"], c["F"], "f32", flags=c["flags"])


def test_adjoint_step_kernel_vs_oracle(case):
    """nu^n = J(f(n))^T P^T nu^{n+1} with f(n) = P f*(n-1): the kernel against
    the oracle's transposed streaming and transposed collision."""
    say("adjoint step kernel vs oracle", case["shape"])
    sim, fl = _sim(case), case["flags"]
    f_to_grid(sim, case["fn"], flags=fl)
    fprev = grid_to_f(sim)  # the FP32-rounded f*(n-1) the kernel sees
    nu1 = to_nu_grid(sim, case["nu1"], fl)
    nu0 = torch.zeros_like(nu1)
    part = torch.zeros(sim.adj_partials_bytes // 8, dtype=torch.float64, device="cuda")
    A.lbm_adjoint_step(sim.ctx, P(sim.grids[sim.current]), P(nu1), P(nu0), P(part))
    dF = torch.empty(3, dtype=torch.float64, device="cuda")
    A.lbm_adjoint_finish_dF(sim.ctx, P(part), P(dF))
    torch.cuda.synchronize()
    lam = O.stream_transpose(case["nu1"], fl)
    ref, dF_ref = O.adjoint_collide(O.stream(fprev, fl), lam, case["tau"], case["F"], fl)
    got = from_nu_grid(sim, nu0, fl)
    e = rel_linf(got, ref)
    eF = np.abs(dF.cpu().numpy() - dF_ref).max() / np.abs(dF_ref).max()
    say(f"  nu rel L-inf {e:.2e}, dL/dF rel {eF:.2e}")
    assert e <= 1e-5 and eF <= 1e-5


def test_adjoint_seed_and_init_kernels_vs_oracle(case):
    """Seed: nu^T = J(f(T))^T lambda^T with lambda^T from dL/drho_T, dL/du_T
    (f(T) = P f*(T-1); the oracle forms lambda^T from f*(T)) and the dL/dF
    terms of both; init: dL/du0 from lambda^0 = P^T nu^1."""
    say("adjoint seed/init kernels vs oracle")
    sim, fl = _sim(case), case["flags"]
    f_to_grid(sim, case["fn"], flags=fl)
    fprev = grid_to_f(sim)
    rng = np.random.default_rng(8)
    shape = case["shape"]
    gr, gu = _f32(rng.standard_normal(shape)), _f32(rng.standard_normal((3,) + shape))
    nu = torch.zeros(sim.grid_bytes // 4, dtype=torch.float32, device="cuda")
    part = torch.zeros(sim.adj_partials_bytes // 8, dtype=torch.float64, device="cuda")
    grt, gut = torch.from_numpy(gr).float().cuda(), torch.from_numpy(gu).float().cuda()
    A.lbm_adjoint_seed(sim.ctx, P(sim.grids[sim.current]), P(grt), P(gut), P(nu), P(part))
    dF = torch.empty(3, dtype=torch.float64, device="cuda")
    A.lbm_adjoint_finish_dF(sim.ctx, P(part), P(dF))
    tau, F = case["tau"], case["F"]
    lam_ref, dF1 = O.adjoint_seed(O.step(fprev, tau, F, fl), gr, gu, F, fl)
    nu_ref, dF2 = O.adjoint_collide(O.stream(fprev, fl), lam_ref, tau, F, fl)
    torch.cuda.synchronize()
    e = rel_linf(from_nu_grid(sim, nu, fl), nu_ref)
    eF = np.abs(dF.cpu().numpy() - (dF1 + dF2)).max() / np.abs(dF1 + dF2).max()
    say(f"  seed: nu rel L-inf {e:.2e}, dL/dF rel {eF:.2e}")
    assert e <= 1e-5 and eF <= 1e-5
    # init: dL/du0 from lambda^0 = P^T nu^1 at (rho0 = 1, u0)
    nu1 = to_nu_grid(sim, case["nu1"], fl)
    u0t = torch.from_numpy(case["u0"]).float().cuda()
    du0 = torch.empty((3,) + shape, dtype=torch.float32, device="cuda")
    A.lbm_adjoint_init(sim.ctx, P(nu1), None, P(u0t), P(du0))
    ref, _ = O.adjoint_init(O.stream_transpose(case["nu1"], fl), case["u0"], fl)
    torch.cuda.synchronize()
    assert rel_linf(du0.double().cpu().numpy(), ref) <= 1e-6


def _gpu_grad(u0, target, F, flags, tau, steps, k, steps_per_pass=0):
    u0t = torch.from_numpy(u0).float().cuda().requires_grad_(True)
    g = torch.tensor(F, dtype=torch.float64, requires_grad=True)
    rho, u = rollout(u0t, g, steps=steps, tau=tau, flags=flags, checkpoint_every=k,
                     steps_per_pass=steps_per_pass)
    fl = torch.ones(u0.shape[1:], dtype=torch.bool, device="cuda") if flags is None else \
        torch.from_numpy((flags & 1) == 0).cuda()
    tt = torch.from_numpy(target).float().cuda()
    loss = ((u - tt) ** 2)[:, fl].mean()
    loss.backward()
    return u0t.grad.double().cpu().numpy(), g.grad.cpu().numpy(), float(loss)


def test_rollout_gradient_vs_oracle_adjoint():
    """16^3 with solids and no-force cells, 30 steps, k = 7."""
    n, tau, steps = 16, 0.6, 30
    shape = (n, n, n)
    say("rollout gradient vs oracle adjoint", shape)
    flags = I.random_flags(shape, 13, solid_fraction=0.1, noforce_fraction=0.1)
    u0 = _f32(I.smooth_field(n, 2024, amplitude=0.02, modes=4))
    u0[:, flags & 1 == 1] = 0
    target = _f32(I.smooth_field(n, 7, amplitude=0.02, modes=4))
    F = np.array([1e-4, -5e-5, 2e-5])
    du0, dF, _ = _gpu_grad(u0, target, F, flags, tau, steps, 7)
    du0_ref, dF_ref = rollout_grad(u0, F, flags, tau, steps, target)
    e_u, e_F = rel_linf(du0, du0_ref), np.abs(dF - dF_ref).max() / np.abs(dF_ref).max()
    say(f"  dL/du0 rel L-inf {e_u:.2e}, dL/dg rel {e_F:.2e}")
    assert e_u <= 1e-4 and e_F <= 1e-4


def test_rollout_gradient_vs_central_differences():
    """Periodic 32^3 copy of the differentiable workload: smooth u0
    (amplitude 0.02), g = (1e-6, 0, 0), tau = 0.6, its 400 steps, k = 20:
    directional derivatives along 4 smooth directions and each force
    component against FP64 central differences of the oracle (eps = 1e-4 on
    u0, 1e-6 on g); bar 1e-4 relative."""
    n, tau, steps = 32, 0.6, 400
    say("rollout gradient vs central differences, 32^3", steps, "steps")
    u0 = _f32(I.smooth_field(n, 2024, amplitude=0.02))
    target = _f32(I.smooth_field(n, 7, amplitude=0.02))
    F = np.array([1e-6, 0.0, 0.0])
    du0, dF, _ = _gpu_grad(u0, target, F, None, tau, steps, 20)
    for s in (101, 102, 103, 104):
        v = I.smooth_field(n, s, amplitude=1.0)
        eps = 1e-4
        fd = (rollout_loss(u0 + eps * v, F, None, tau, steps, target)
              - rollout_loss(u0 - eps * v, F, None, tau, steps, target)) / (2 * eps)
        ad = float((du0 * v).sum())
        say(f"  direction {s}: adjoint {ad:.6e}  FD {fd:.6e}  rel {abs(ad - fd) / abs(fd):.2e}")
        assert abs(ad - fd) <= 1e-4 * abs(fd)
    for a in range(3):
        d = np.zeros(3)
        d[a] = 1e-6
        fd = (rollout_loss(u0, F + d, None, tau, steps, target)
              - rollout_loss(u0, F - d, None, tau, steps, target)) / 2e-6
        say(f"  g[{a}]: adjoint {dF[a]:.6e}  FD {fd:.6e}")
        assert abs(dF[a] - fd) <= 1e-4 * abs(fd)


@pytest.mark.timeout(600)
def test_rollout_gradient_at_workload_size_vs_central_difference():
    """The differentiable workload as the bench times it: periodic 128^3,
    smooth u0 (seed 2024, amplitude 0.02), target seed 7, g = (1e-6, 0, 0),
    tau = 0.6, 400 steps, checkpoints every 20.  One directional derivative
    of the GPU gradient (a smooth direction, seed 101) against an FP64
    central difference of the oracle (eps = 1e-4), and the force gradient's
    x component against one at eps = 1e-6; bar 1e-4 relative."""
    n, tau, steps = 128, 0.6, 400
    say("rollout gradient at 128^3 x 400 steps vs one central difference each")
    u0 = _f32(I.smooth_field(n, 2024, amplitude=0.02))
    target = _f32(I.smooth_field(n, 7, amplitude=0.02))
    F = np.array([1e-6, 0.0, 0.0])
    du0, dF, _ = _gpu_grad(u0, target, F, None, tau, steps, 20)
    torch.cuda.empty_cache()
    v = I.smooth_field(n, 101, amplitude=1.0)
    eps = 1e-4
    losses = []
    for sgn in (1, -1):
        say(f"  oracle rollout u0 {'+' if sgn > 0 else '-'} eps v ...")
        losses.append(rollout_loss(u0 + sgn * eps * v, F, None, tau, steps, target))
    fd = (losses[0] - losses[1]) / (2 * eps)
    ad = float((du0 * v).sum())
    say(f"  direction 101: adjoint {ad:.6e}  FD {fd:.6e}  rel {abs(ad - fd) / abs(fd):.2e}")
    assert abs(ad - fd) <= 1e-4 * abs(fd)
    d = np.array([1e-6, 0.0, 0.0])
    losses = []
    for sgn in (1, -1):
        say(f"  oracle rollout g {'+' if sgn > 0 else '-'} eps ...")
        losses.append(rollout_loss(u0, F + sgn * d, None, tau, steps, target))
    fdg = (losses[0] - losses[1]) / 2e-6
    say(f"  g[0]: adjoint {dF[0]:.6e}  FD {fdg:.6e}  rel {abs(dF[0] - fdg) / abs(fdg):.2e}")
    assert abs(dF[0] - fdg) <= 1e-4 * abs(fdg)


def test_checkpoint_spacing_gives_identical_gradients():
    n, tau, steps = 32, 0.6, 40
    say("checkpoint spacing 1 / 7 / 20 / 40")
    flags = I.random_flags((n, n, n), 3, solid_fraction=0.05)
    u0 = _f32(I.smooth_field(n, 5, amplitude=0.02, modes=4))
    u0[:, flags & 1 == 1] = 0
    target = _f32(I.smooth_field(n, 6, amplitude=0.02, modes=4))
    F = np.array([1e-5, 0, 0])
    ref = _gpu_grad(u0, target, F, flags, tau, steps, 1)
    for k in (7, 20, 40):
        got = _gpu_grad(u0, target, F, flags, tau, steps, k)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), k


def test_forward_in_fused_pairs_gives_identical_gradients():
    """The forward sweep in fused pairs of steps (even and odd segment
    lengths: k = 7 ends every segment with a single step) reaches the same
    states bit for bit, so the gradients and the loss are identical."""
    n, tau, steps = 32, 0.6, 41
    say("rollout forward in fused pairs, k = 7 / 20")
    flags = I.random_flags((n, n, n), 4, solid_fraction=0.05, noforce_fraction=0.1)
    u0 = _f32(I.smooth_field(n, 8, amplitude=0.02, modes=4))
    u0[:, flags & 1 == 1] = 0
    target = _f32(I.smooth_field(n, 9, amplitude=0.02, modes=4))
    F = np.array([1e-5, -2e-6, 0])
    for k in (7, 20):
        ref = _gpu_grad(u0, target, F, flags, tau, steps, k)
        got = _gpu_grad(u0, target, F, flags, tau, steps, k, steps_per_pass=2)
        assert got[2] == ref[2], k
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), k


def test_fused_recomputation_gives_identical_gradients(monkeypatch):
    """The reverse sweep's recomputation in fused pairs (lbm_step2_from,
    used from 256^3 on) reaches the same states, so the same gradients: the
    threshold lowered to force it on a small box, odd and even segments."""
    from paper_1112_0850_amd import lbm as L
    n, tau, steps = 24, 0.6, 23
    flags = I.random_flags((n, n, n), 14, solid_fraction=0.08, noforce_fraction=0.1)
    u0 = _f32(I.smooth_field(n, 15, amplitude=0.02, modes=3))
    u0[:, flags & 1 == 1] = 0
    target = _f32(I.smooth_field(n, 16, amplitude=0.02, modes=3))
    F = np.array([2e-5, 0, -1e-5])
    for k, spp in ((6, 0), (9, 0), (6, 2)):  # spp = 2: the link mask in the recomputation
        monkeypatch.setattr(L, "FUSED_RECOMPUTE_MIN_CELLS", 1 << 40)
        ref = _gpu_grad(u0, target, F, flags, tau, steps, k)
        monkeypatch.setattr(L, "FUSED_RECOMPUTE_MIN_CELLS", 0)
        got = _gpu_grad(u0, target, F, flags, tau, steps, k, steps_per_pass=spp)
        assert got[2] == ref[2] and np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), k

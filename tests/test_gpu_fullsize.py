"""Parity at the benchmark's full size and launch configuration: the 512^3
porous box (10% spheres, seed 12345, tau = 0.55, g_x = 1e-6) and the 512^3
lid-driven cavity (moving-wall kernel), one fused step checked cell by cell
on sampled cells, where the oracle recomputes each sampled cell from its
3^3 neighbourhood of the previous state; and the adjoint kernel at the
rollout's 128^3 size, checked on 5^3 neighbourhoods."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1112_0850_amd import _abi as A
from paper_1112_0850_amd import inputs as I
from paper_1112_0850_amd.lbm import LBM
from tests.gpu_util import W, say

pytestmark = pytest.mark.gpu
N = 512
TAU, F = 0.55, (1e-6, 0.0, 0.0)


@pytest.fixture(scope="module")
def geometry():
    flags = I.sphere_pack((N, N, N), 0.10, seed=12345)
    u0 = I.shear_waves((N, N, N), seed=21, amplitude=0.02)
    u0[:, flags & 1 == 1] = 0
    return flags, torch.from_numpy(u0)


def _crop(view, z, y, x, r, nz, ny, nx):
    """[19, 2r+1, 2r+1, 2r+1] periodic crop of a [19, nz, ny, xs] device view."""
    zi = torch.tensor([(z + d) % nz for d in range(-r, r + 1)], device=view.device)
    yi = torch.tensor([(y + d) % ny for d in range(-r, r + 1)], device=view.device)
    xi = torch.tensor([(x + d) % nx for d in range(-r, r + 1)], device=view.device)
    return view[:, zi[:, None, None], yi[None, :, None], xi[None, None, :]]


def _fcrop(flags, z, y, x, r):
    n = flags.shape
    zi = [(z + d) % n[0] for d in range(-r, r + 1)]
    yi = [(y + d) % n[1] for d in range(-r, r + 1)]
    xi = [(x + d) % n[2] for d in range(-r, r + 1)]
    return np.ascontiguousarray(flags[np.ix_(zi, yi, xi)])


@pytest.mark.parametrize("storage,s", [("f32", 0), ("f16", 12), ("bf16", 0), ("f64", 0), ("f32x", 0)])
def test_sampled_step_at_full_size(geometry, storage, s):
    flags, u0 = geometry
    say(f"full size {N}^3 porous, {storage}: sampled one-step parity")
    sim = LBM((N, N, N), TAU, F, storage, flags=flags, u0=u0, f16_scale_log2=s)
    rng = np.random.default_rng(2024)
    fluid = np.flatnonzero((flags & 1 == 0).ravel())
    _sampled_step(sim, flags, storage, s, rng.choice(fluid, size=256, replace=False), TAU, F, None)


@pytest.mark.parametrize("storage,s", [("f32", 0), ("f16", 12)])
def test_sampled_incompressible_step_at_full_size(geometry, storage, s):
    """The bench's incompressible-equilibrium legs: the 512^3 porous box with
    the He-Luo equilibrium, sampled one-step parity."""
    flags, u0 = geometry
    say(f"full size {N}^3 porous, incompressible, {storage}: sampled one-step parity")
    sim = LBM((N, N, N), TAU, F, storage, flags=flags, u0=u0, f16_scale_log2=s,
              equilibrium="incompressible")
    rng = np.random.default_rng(2025)
    fluid = np.flatnonzero((flags & 1 == 0).ravel())
    _sampled_step(sim, flags, storage, s, rng.choice(fluid, size=256, replace=False), TAU, F, None,
                  incompressible=True)


@pytest.mark.parametrize("storage,s", [("f32", 0), ("f16", 12)])
def test_split_design_matches_fused_at_full_size(geometry, storage, s):
    """The bench's split-design legs (separate obstacle kernel) against the
    fused step on the 512^3 porous box: identical fluid-cell bits after a
    few steps (the solid cells' slots differ by design: bounce-back values
    there, markers in the fused grids)."""
    flags, u0 = geometry
    say(f"full size {N}^3 porous, {storage}: split design == fused")
    fused = LBM((N, N, N), TAU, F, storage, flags=flags, u0=u0, f16_scale_log2=s).step(5)
    split = LBM((N, N, N), TAU, F, storage, flags=flags, u0=u0, f16_scale_log2=s,
                obstacle_kernel=1).step(5)
    torch.cuda.synchronize()
    fluid = torch.from_numpy((flags & 1) == 0).cuda()
    a, b = fused.populations()[..., :N], split.populations()[..., :N]
    for i in range(19):
        assert torch.equal(a[i][fluid], b[i][fluid]), i
    del fused, split, a, b
    torch.cuda.empty_cache()


def test_pull_copy_probe_at_full_size():
    """The pull-copy probe as the bench times it (512^3 FP32 layout): sampled
    cells of dst equal src at x - c_i (periodic)."""
    from tests import lattice_ref as R
    say(f"full size {N}^3 pull-copy probe, sampled")
    e = R.e_w_opp()[0]
    sim = LBM((N, N, N), TAU, F, "f32")
    src, dst = sim.new_grid(), sim.new_grid().zero_()
    sv = sim.grid_view(src)
    sv.copy_(torch.rand(sv.shape, device="cuda", dtype=torch.float32))
    sim.pull_copy(src, dst)
    torch.cuda.synchronize()
    dv = sim.grid_view(dst)
    rng = np.random.default_rng(5)
    zyx = rng.integers(0, N, size=(512, 3))
    zyx[:8] = [(0, 0, 0), (N - 1, N - 1, N - 1), (0, N - 1, 0), (N - 1, 0, N - 1),
               (0, 0, N - 1), (N - 1, N - 1, 0), (N // 2, 0, 0), (0, N // 2, N - 1)]
    for i in range(19):
        z, y, x = (torch.from_numpy(zyx[:, k]).cuda() for k in range(3))
        zs, ys, xs = (z - int(e[i, 2])) % N, (y - int(e[i, 1])) % N, (x - int(e[i, 0])) % N
        assert torch.equal(dv[i, z, y, x], sv[i, zs, ys, xs]), i
    del sim, src, dst, sv, dv
    torch.cuda.empty_cache()


CAVITY_TAU, CAVITY_U = 0.55, 0.05
CAVITY_TAU, CAVITY_U = 0.55, 0.05


@pytest.mark.parametrize("storage,s", [("f32", 0), ("f16", 10)])
def test_sampled_cavity_step_at_full_size(storage, s):
    """512^3 lid-driven cavity (top plane moving with (0.05, 0, 0)), after
    40 steps from rest: cells under the lid (edges and corners included),
    beside the side walls and at random."""
    say(f"full size {N}^3 lid-driven cavity, {storage}: sampled one-step parity")
    flags = I.cavity_flags((N, N, N))
    sim = LBM((N, N, N), CAVITY_TAU, (0, 0, 0), storage, flags=flags, wall_u=(CAVITY_U, 0, 0),
              f16_scale_log2=s)
    sim.step(36)
    rng = np.random.default_rng(77)
    zyx = [(N - 2, 1, 1), (N - 2, N - 2, N - 2), (N - 2, 1, N - 2), (N - 2, N // 2, 1),
           (N - 2, N // 2, N // 2), (1, 1, 1), (N // 2, 1, N // 2)]
    zyx += [(N - 2, int(a), int(b)) for a, b in rng.integers(1, N - 1, size=(60, 2))]
    zyx += [tuple(int(v) for v in rng.integers(1, N - 1, size=3)) for _ in range(60)]
    cells = [(z * N + y) * N + x for z, y, x in zyx]
    _sampled_step(sim, flags, storage, s, cells, CAVITY_TAU, (0, 0, 0), (CAVITY_U, 0, 0))


def _sampled_step(sim, flags, storage, s, cells, tau, F, wall_u, extra=3, incompressible=False):
    """`extra` more steps, then one: each sampled fluid cell of the last step
    against the oracle's step of its 3^3 neighbourhood, read from the state
    before that step (no copy of the grid is made, so this runs at sizes
    where only the two lattices fit)."""
    nz, ny, nx = sim.shape
    sim.step(extra)
    torch.cuda.synchronize()
    pv = sim.populations()
    scale = 2.0 ** s
    crops = []
    for c in cells:
        z, rem = divmod(int(c), ny * nx)
        y, x = divmod(rem, nx)
        g = _crop(pv, z, y, x, 1, nz, ny, nx).double().cpu().numpy() / scale
        crops.append((z, y, x, g, _fcrop(flags, z, y, x, 1)))
    sim.step(1)
    torch.cuda.synchronize()
    cv = sim.populations()
    worst = 0.0
    gmax = 0.0
    for z, y, x, g, fl in crops:
        f = g + W[:, None, None, None]
        f[:, fl & 1 == 1] = 0
        ref = O.step(f, tau, F, fl, n=1, wall_u=wall_u,
                     incompressible=incompressible)[:, 1, 1, 1] - W
        got = cv[:, z, y, x].double().cpu().numpy() / scale
        if storage in ("f32", "f32x"):
            err = np.abs(got - ref)
            bound = 1e-6 * np.abs(ref).max() + 1e-12
        elif storage == "f64":
            # the oracle rounds f = g + w (|f| ~ 1/3) through ~50 operations:
            # an absolute floor of ~50 ulp(1)/2, beside the relative bound
            err = np.abs(got - ref)
            bound = 1e-13 * np.abs(ref).max() + 1e-14
        else:
            if storage == "f16":
                ulp = np.spacing(np.abs(ref * scale).astype(np.float16)).astype(np.float64) / scale
            else:  # bfloat16: 8 significant bits
                ulp = 2.0 ** (np.floor(np.log2(np.maximum(np.abs(ref), 1e-38))) - 7)
            err = np.abs(got - ref) - 0.5 * ulp
            bound = 2e-6 * np.abs(ref).max()
        worst = max(worst, float(err.max()))
        gmax = max(gmax, float(np.abs(ref).max()))
        assert (err <= bound).all(), (storage, z, y, x, err.max(), bound)
    say(f"  worst excess error {worst:.2e} (offset scale {gmax:.2e})")
    del sim
    torch.cuda.empty_cache()


@pytest.mark.parametrize("storage,n", [("f32", 768), ("f64", 640)])
def test_sampled_step_large_boxes(storage, n):
    """The large-box workloads as timed (5% spheres r 4-12, seed 777,
    tau 0.55, g_x 1e-6): 68.9 GB FP32 at 768^3, 79.7 GB FP64 at 640^3."""
    say(f"large box {n}^3 {storage}: sampled one-step parity")
    flags = I.sphere_pack((n, n, n), 0.05, seed=777)
    u0 = I.shear_waves((n, n, n), seed=5, amplitude=0.02)
    u0[:, flags & 1 == 1] = 0
    sim = LBM((n, n, n), TAU, F, storage, flags=flags, u0=torch.from_numpy(u0))
    del u0
    rng = np.random.default_rng(768)
    fluid = np.flatnonzero((flags & 1 == 0).ravel())
    _sampled_step(sim, flags, storage, 0, rng.choice(fluid, size=128, replace=False), TAU, F, None)


def test_sampled_step_at_maximum_size():
    """The largest FP32 box the 32-bit lane offsets allow: 1023^3 (x stride
    1024: one direction array is 4,286,582,784 bytes, just under 4 GiB), a
    channel with walls at y = 0 and y = 1022; cells sampled near the far end
    of the arrays, where the offsets are largest, and at random."""
    n = 1023
    say(f"maximum size {n}^3 f32: sampled one-step parity")
    p = A.params((n, n, n), TAU, F)
    xs, ds, gb, _, _ = A.lbm_query(p)
    assert xs == 1024 and ds == n * n * xs + 64 and 19 * ds * 4 <= gb and n * n * xs * 4 < 2 ** 32
    flags = I.channel_flags((n, n, n))
    sim = LBM((n, n, n), TAU, F, "f32", flags=flags)
    rng = np.random.default_rng(1023)
    zyx = [(n - 1, n - 2, n - 1), (n - 1, 1, 0), (n - 2, n - 2, n - 2), (0, 1, 0), (n // 2, n - 2, 5)]
    zyx += [(int(z), int(y), int(x)) for z, y, x in
            zip(rng.integers(0, n, 60), rng.integers(1, n - 1, 60), rng.integers(0, n, 60))]
    cells = [(z * n + y) * n + x for z, y, x in zyx]
    _sampled_step(sim, flags, "f32", 0, cells, TAU, F, None, extra=2)


def test_sampled_adjoint_step_at_rollout_size():
    """The pull-form adjoint step at the rollout's 128^3 size: nu^n at sampled
    cells against the oracle's transposed streaming and transposed collision
    on the cell's 5^3 neighbourhood (periodic crops; the centre depends on
    its 3^3 neighbours only)."""
    n = 128
    say(f"adjoint kernel at {n}^3: sampled parity on 5^3 neighbourhoods")
    u0 = torch.from_numpy(I.smooth_field(n, 2024, amplitude=0.02))
    sim = LBM((n, n, n), 0.6, (1e-6, 0, 0), "f32", u0=u0)
    sim.step(5)
    rng = np.random.default_rng(6)
    nu1 = torch.zeros(sim.grid_bytes // 4, dtype=torch.float32, device="cuda")
    v1 = sim.grid_view(nu1)
    v1[..., :n].copy_(torch.from_numpy(rng.standard_normal((19, n, n, n)).astype(np.float32)))
    nu0 = torch.zeros_like(nu1)
    part = torch.zeros(sim.adj_partials_bytes // 8, dtype=torch.float64, device="cuda")
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    A.lbm_adjoint_step(sim.ctx, P(sim.grids[sim.current]), P(nu1), P(nu0), P(part))
    torch.cuda.synchronize()
    v0 = sim.grid_view(nu0)
    fv = sim.populations()
    worst = 0.0
    zyx = [(0, 0, 0), (n - 1, n - 1, n - 1), (0, n - 1, 63), (n - 1, 0, 64)]
    zyx += [tuple(int(v) for v in rng.integers(0, n, size=3)) for _ in range(60)]
    for z, y, x in zyx:
        f = _crop(fv, z, y, x, 2, n, n, n).double().cpu().numpy() + W[:, None, None, None]
        l1 = _crop(v1, z, y, x, 2, n, n, n).double().cpu().numpy()
        ref, _ = O.adjoint_collide(O.stream(f), O.stream_transpose(l1), 0.6, (1e-6, 0, 0))
        got = v0[:, z, y, x].double().cpu().numpy()
        e = np.abs(got - ref[:, 2, 2, 2]).max() / np.abs(ref[:, 2, 2, 2]).max()
        worst = max(worst, e)
        assert e <= 1e-5, (z, y, x, e)
    say(f"  worst relative error {worst:.2e}")


@pytest.mark.parametrize("storage,s", [("f32", 0), ("f16", 12)])
def test_sampled_step_unpadded_500(storage, s):
    """The domain sweep's unpadded layout at one of its sizes (x_align = 1:
    rows 500 cells apart, so rows start at every 16-byte offset and the
    64-cell segments straddle row ends): 500^3 porous box (10% spheres,
    seed 12345), sampled one-step parity, rows near both ends included."""
    n = 500
    say(f"unpadded {n}^3 porous, {storage}: sampled one-step parity")
    flags = I.sphere_pack((n, n, n), 0.10, seed=12345)
    u0 = I.shear_waves((n, n, n), seed=8, amplitude=0.02)
    u0[:, flags & 1 == 1] = 0
    sim = LBM((n, n, n), TAU, F, storage, flags=flags, u0=torch.from_numpy(u0), x_align=1,
              f16_scale_log2=s)
    assert sim.x_stride == n
    del u0
    rng = np.random.default_rng(500)
    fluid = (flags & 1) == 0
    zyx = [(z, y, x) for z, y, x in [(0, 0, 0), (n - 1, n - 1, n - 1), (3, 7, n - 1), (9, 2, 0),
                                     (n - 1, 0, 447), (1, n - 1, 448), (5, 5, 63), (6, 6, 64)]
           if fluid[z, y, x]]
    cells = [(z * n + y) * n + x for z, y, x in zyx]
    cells += list(rng.choice(np.flatnonzero(fluid.ravel()), size=160, replace=False))
    _sampled_step(sim, flags, storage, s, cells, TAU, F, None)

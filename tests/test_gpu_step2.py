"""The two-step pass (steps_per_pass = 2: pairs of steps fused into one
temporally blocked kernel that keeps the intermediate level on chip; resting
walls through the link mask, moving walls and oversized grids through the
markers) gives the same bits as single steps -- every storage, resting walls
(sparse and dense), moving walls, moving-wall flags at zero wall velocity,
a change of the flags after some steps,
no-force cells, both equilibria, ragged and degenerate shapes, several z
chunks, the unpadded layout, graph replays, odd step counts -- and the
oracle's result within the FP32 bar; at the benchmark's full size as well."""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1112_0850_amd import _abi as A
from paper_1112_0850_amd import inputs as I
from paper_1112_0850_amd.lbm import LBM
from tests.gpu_util import check_solids, rel_linf, say

pytestmark = pytest.mark.gpu

STORAGES = ["f32", "f16", "bf16", "f64", "f32x"]


def _pair(shape, tau, F, storage, n, **kw):
    s = 10 if storage == "f16" else 0
    one = LBM(shape, tau, F, storage, f16_scale_log2=s, **kw).step(n)
    two = LBM(shape, tau, F, storage, f16_scale_log2=s, steps_per_pass=2, **kw).step(n)
    torch.cuda.synchronize()
    return one, two


def _same(one, two):
    """Equal bytes in the current grids; on a difference, report where."""
    assert one.t == two.t
    a, b = one.grids[one.current], two.grids[two.current]
    if torch.equal(a, b):
        return True
    nz, ny, nx = one.shape
    va, vb = one.populations()[..., :nx], two.populations()[..., :nx]
    ia = va.contiguous().view(torch.int16 if va.element_size() == 2 else
                              (torch.int32 if va.element_size() == 4 else torch.int64))
    ib = vb.contiguous().view(ia.dtype)
    d = (ia != ib).nonzero().cpu().numpy()
    say(f"  {len(d)} differing elements; first (i, z, y, x): {d[:8].tolist()}")
    say(f"  per direction: {np.bincount(d[:, 0], minlength=19).tolist()}")
    return False


def _u0(shape, seed, amp=0.03):
    rng = np.random.default_rng(seed)
    return torch.from_numpy(amp * (rng.random((3,) + shape) - 0.5)).float()


CASES = {
    # name: (shape, kwargs)
    "ragged_porous": ((7, 11, 100), "flags"),
    "periodic": ((9, 16, 128), None),
    "moving_walls": ((10, 12, 70), "moving"),
    "z_chunks": ((300, 9, 70), "flags"),
    "single_cell": ((1, 1, 1), None),
    "thin_slab": ((1, 5, 1), None),
    "narrow": ((3, 2, 17), "flags"),
    "dense_solids": ((11, 13, 90), "dense"),
    "tiny_porous": ((2, 1, 3), "tiny"),  # every pull wraps onto the box itself
    "moving_flags_at_rest": ((10, 12, 70), "moving_at_rest"),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("storage", STORAGES)
def test_two_step_pass_is_bit_identical(storage, case):
    shape, geo = CASES[case]
    say("two-step pass vs single steps", storage, case, shape)
    kw = dict(u0=_u0(shape, 3))
    if geo == "flags":
        kw["flags"] = I.random_flags(shape, 9, solid_fraction=0.2, noforce_fraction=0.15)
    elif geo == "moving":
        fl = I.random_flags(shape, 10, solid_fraction=0.15, noforce_fraction=0.1) | I.cavity_flags(shape)
        kw.update(flags=fl, wall_u=(0.04, -0.01, 0.02))
    elif geo == "tiny":  # one solid cell, one no-force cell
        fl = np.zeros(shape, dtype=np.uint8)
        fl[0, 0, 1] = I.FLAG_SOLID
        fl[1, 0, 2] = I.FLAG_NOFORCE
        kw["flags"] = fl
    elif geo == "dense":  # most links blocked
        kw["flags"] = I.random_flags(shape, 19, solid_fraction=0.6, noforce_fraction=0.1)
    elif geo == "moving_at_rest":  # moving-wall flags, zero wall velocity: resting walls
        kw["flags"] = (I.random_flags(shape, 20, solid_fraction=0.15, noforce_fraction=0.1)
                       | I.cavity_flags(shape))
    if "flags" in kw:
        kw["u0"][:, torch.from_numpy(kw["flags"] & 1 == 1)] = 0
    for eq in ("qian", "incompressible"):
        one, two = _pair(shape, 0.63, (2e-5, -1e-5, 3e-5), storage, 9, equilibrium=eq, **kw)
        assert _same(one, two), eq
        if "flags" in kw:
            check_solids(two, kw["flags"])


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_two_step_pass_unpadded_and_without_force(storage):
    shape = (6, 10, 65)
    say("two-step pass, unpadded rows, no force", storage)
    fl = I.random_flags(shape, 4, solid_fraction=0.2)
    one, two = _pair(shape, 0.7, (0, 0, 0), storage, 8, flags=fl, x_align=1, u0=_u0(shape, 5))
    assert two.x_stride == 65 and _same(one, two)


@pytest.mark.parametrize("storage", ["f32", "f16", "f64"])
def test_two_step_pass_follows_changed_flags(storage):
    """Cells turned solid after some steps (the flags changed in place, then
    lbm_refresh_solids): the pass's link mask follows the new geometry, and
    pairs still equal single steps bit for bit."""
    shape = (12, 14, 70)
    say("two-step pass after a change of the flags", storage)
    fl = I.random_flags(shape, 21, solid_fraction=0.1, noforce_fraction=0.1)
    u0 = _u0(shape, 22)
    u0[:, torch.from_numpy(fl & 1 == 1)] = 0
    s = 10 if storage == "f16" else 0
    sims = [LBM(shape, 0.6, (1e-5, 0, 0), storage, flags=fl, u0=u0, f16_scale_log2=s,
                steps_per_pass=spp).step(4) for spp in (0, 2)]
    more = (I.random_flags(shape, 23, solid_fraction=0.05) & 1).astype(np.uint8)
    for sim in sims:
        sim.flags |= torch.from_numpy(more).cuda()
        sim.refresh_solids()
        sim.step(6)
    torch.cuda.synchronize()
    assert _same(*sims)
    check_solids(sims[1], fl | more)


def test_link_mask_content():
    """The link mask the two-step pass reads, read back from the context's
    scratch (after the reduction's partials): bit i set exactly when the pull
    along c_i comes from a solid cell (periodic), bit 19 SOLID, bit 20
    NOFORCE -- against the same rule written out from the flags in numpy."""
    shape = (7, 9, 70)
    fl = I.random_flags(shape, 31, solid_fraction=0.2, noforce_fraction=0.15)
    sim = LBM(shape, 0.6, (1e-5, 0, 0), "f32", flags=fl, steps_per_pass=2)
    torch.cuda.synchronize()
    cells = int(np.prod(shape))
    off = (1024 * 5 * 8 + 255) // 256 * 256  # the reduction's 1024 x 5 FP64 partials
    got = sim.scratch.view(torch.uint8)[off:off + 4 * cells].view(torch.int32).cpu().numpy()
    got = got.view(np.uint32).reshape(shape)
    e, _, _ = O.lattice()
    solid = (fl & 1) == 1
    want = np.where(solid, 1 << 19, 0).astype(np.uint32) | np.where(fl & 2, 1 << 20, 0).astype(np.uint32)
    for i in range(1, 19):
        cx, cy, cz = (int(v) for v in e[i])
        src = np.roll(solid, (cz, cy, cx), axis=(0, 1, 2))  # solid(x - c_i)
        want |= np.where(src, np.uint32(1 << i), np.uint32(0))
    assert np.array_equal(got, want)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_two_step_pass_with_graph_replays(storage):
    """Graphs of 6 steps (three fused passes: the replay ends on the other
    grid) interleaved with odd eager counts."""
    shape = (8, 9, 70)
    say("two-step pass under graph replays", storage)
    fl = I.random_flags(shape, 6, solid_fraction=0.2, noforce_fraction=0.1)
    s = 10 if storage == "f16" else 0
    ref = LBM(shape, 0.6, (1e-5, 0, 0), storage, flags=fl, u0=_u0(shape, 7), f16_scale_log2=s)
    g = LBM(shape, 0.6, (1e-5, 0, 0), storage, flags=fl, u0=_u0(shape, 7), f16_scale_log2=s,
            steps_per_pass=2).use_graphs(6)
    for n in (6, 3, 12, 1, 6, 5):
        ref.step(n)
        g.step(n)
        torch.cuda.synchronize()
        assert _same(ref, g), n


def test_two_step_pass_porous_parity_vs_oracle():
    """The porous parity case run in pairs: FP32 within 1e-5 of the FP64
    oracle after 100 steps."""
    shape = (64, 64, 64)
    say("two-step pass, porous 64^3 vs oracle")
    flags = I.sphere_pack(shape, 0.10, seed=12345)
    u0 = I.smooth_field(64, 99, amplitude=0.02, modes=4)
    u0[:, flags & 1 == 1] = 0
    u0 = u0.astype(np.float32).astype(np.float64)
    sim = LBM(shape, 0.55, (1e-6, 0, 0), "f32", flags=flags, u0=torch.from_numpy(u0).float(),
              steps_per_pass=2).step(100)
    f = O.step(O.init(shape, flags, None, u0), 0.55, (1e-6, 0, 0), flags, n=100)
    rho, u = sim.macroscopics(f64=True)
    rho_r, u_r = O.macroscopics(f, (1e-6, 0, 0), flags)
    fl = (flags & 1) == 0
    e_rho, e_u = rel_linf(rho.cpu().numpy(), rho_r, fl), rel_linf(u.cpu().numpy(), u_r, fl)
    say(f"  rel L-inf rho {e_rho:.2e}  u {e_u:.2e}")
    assert e_rho <= 1e-5 and e_u <= 1e-5


@pytest.mark.parametrize("storage,s", [("f32", 0), ("f16", 12), ("bf16", 0), ("f64", 0), ("f32x", 0)])
def test_two_step_pass_at_full_size(storage, s):
    """The benchmark's 512^3 porous box (10% spheres, seed 12345, tau 0.55,
    g_x 1e-6) from a sheared start: 6 steps in fused pairs == 6 single steps,
    every byte of the grid."""
    n = 512
    say(f"two-step pass at {n}^3 porous, {storage}")
    flags = I.sphere_pack((n, n, n), 0.10, seed=12345)
    u0 = I.shear_waves((n, n, n), seed=21, amplitude=0.02)
    u0[:, flags & 1 == 1] = 0
    u0 = torch.from_numpy(u0)
    one = LBM((n, n, n), 0.55, (1e-6, 0, 0), storage, flags=flags, u0=u0, f16_scale_log2=s).step(6)
    two = LBM((n, n, n), 0.55, (1e-6, 0, 0), storage, flags=flags, u0=u0, f16_scale_log2=s,
              steps_per_pass=2).step(6)
    torch.cuda.synchronize()
    assert _same(one, two)
    del one, two
    torch.cuda.empty_cache()


@pytest.mark.parametrize("storage,s", [("f32", 0), ("f16", 10)])
def test_two_step_pass_cavity_at_full_size(storage, s):
    n = 512
    say(f"two-step pass at {n}^3 lid-driven cavity, {storage}")
    flags = I.cavity_flags((n, n, n))
    kw = dict(flags=flags, wall_u=(0.05, 0, 0), f16_scale_log2=s)
    one = LBM((n, n, n), 0.55, (0, 0, 0), storage, **kw).step(4)
    two = LBM((n, n, n), 0.55, (0, 0, 0), storage, steps_per_pass=2, **kw).step(4)
    torch.cuda.synchronize()
    assert _same(one, two)
    del one, two
    torch.cuda.empty_cache()


def _sampled_two_steps(sim, flags, cells, tau, F, extra=2, rel=1e-6):
    """`extra` steps, then one fused pass of two: each sampled fluid cell
    against the oracle's two steps of its 5^3 neighbourhood, read from the
    state before the pass (the centre after two steps depends on that
    neighbourhood only; no copy of the grid, so one box fills the GPU)."""
    nz, ny, nx = sim.shape
    sim.step(extra)
    torch.cuda.synchronize()
    pv = sim.populations()
    crops = []
    for c in cells:
        z, rem = divmod(int(c), ny * nx)
        y, x = divmod(rem, nx)
        zi = torch.tensor([(z + d) % nz for d in range(-2, 3)], device=pv.device)
        yi = torch.tensor([(y + d) % ny for d in range(-2, 3)], device=pv.device)
        xi = torch.tensor([(x + d) % nx for d in range(-2, 3)], device=pv.device)
        g = pv[:, zi[:, None, None], yi[None, :, None], xi[None, None, :]].double().cpu().numpy()
        fl = np.ascontiguousarray(flags[np.ix_([(z + d) % nz for d in range(-2, 3)],
                                               [(y + d) % ny for d in range(-2, 3)],
                                               [(x + d) % nx for d in range(-2, 3)])])
        crops.append((z, y, x, g, fl))
    t0 = sim.t
    sim.step(2)
    torch.cuda.synchronize()
    assert sim.t == t0 + 2
    cv = sim.populations()
    _, w, _ = O.lattice()
    worst = 0.0
    for z, y, x, g, fl in crops:
        f = g + w[:, None, None, None]
        f[:, fl & 1 == 1] = 0
        ref = O.step(f, tau, F, fl, n=2)[:, 2, 2, 2] - w
        got = cv[:, z, y, x].double().cpu().numpy()
        err = np.abs(got - ref)
        bound = rel * np.abs(ref).max() + 1e-12 * rel / 1e-6
        worst = max(worst, float(err.max()))
        assert (err <= bound).all(), (z, y, x, err.max(), bound)
    say(f"  worst error {worst:.2e}")


def test_two_step_pass_large_box():
    """The large-box workload (768^3, 5% spheres r 4-12, seed 777, tau 0.55,
    g_x 1e-6; 68.9 GB FP32) in fused pairs: sampled cells against the
    oracle."""
    n = 768
    say(f"two-step pass at {n}^3 porous f32: sampled parity")
    flags = I.sphere_pack((n, n, n), 0.05, seed=777)
    u0 = I.shear_waves((n, n, n), seed=5, amplitude=0.02)
    u0[:, flags & 1 == 1] = 0
    sim = LBM((n, n, n), 0.55, (1e-6, 0, 0), "f32", flags=flags, u0=torch.from_numpy(u0),
              steps_per_pass=2)
    del u0
    rng = np.random.default_rng(7682)
    fluid = np.flatnonzero((flags & 1 == 0).ravel())
    _sampled_two_steps(sim, flags, rng.choice(fluid, size=96, replace=False), 0.55, (1e-6, 0, 0))
    del sim
    torch.cuda.empty_cache()


def test_two_step_pass_fp64_large_box():
    """The large-box workload's FP64 case (640^3, 5% spheres r 4-12, seed
    777, tau 0.55, g_x 1e-6; 79.7 GB) in fused pairs, where the link mask's
    pulls address two direction arrays of 2.1 GB from one base (offsets up
    to 4.19 GB): cells at the far end of the arrays and at random against
    the oracle, to 1e-12."""
    n = 640
    say(f"two-step pass at {n}^3 porous f64: sampled parity")
    flags = I.sphere_pack((n, n, n), 0.05, seed=777)
    u0 = I.shear_waves((n, n, n), seed=6, amplitude=0.02)
    u0[:, flags & 1 == 1] = 0
    sim = LBM((n, n, n), 0.55, (1e-6, 0, 0), "f64", flags=flags, u0=torch.from_numpy(u0),
              steps_per_pass=2)
    del u0
    rng = np.random.default_rng(6402)
    fluid = flags & 1 == 0
    far = [(z, y, x) for z in (n - 1, n - 2) for y in (n - 1, n - 3) for x in (n - 1, 0, 63)
           if fluid[z, y, x]]
    cells = [(z * n + y) * n + x for z, y, x in far]
    cells += list(rng.choice(np.flatnonzero(fluid.ravel()), size=64, replace=False))
    _sampled_two_steps(sim, flags, cells, 0.55, (1e-6, 0, 0), rel=1e-12)
    del sim
    torch.cuda.empty_cache()


def test_two_step_pass_at_maximum_size():
    """The largest FP32 box the 32-bit offsets allow (1023^3, one direction
    array just under 4 GiB), a channel with walls at y = 0 and y = 1022, in
    fused pairs: cells near the far end of the arrays, where the byte offsets
    are largest, at the tile and chunk edges, and at random."""
    n = 1023
    say(f"two-step pass at {n}^3 channel f32: sampled parity")
    flags = I.channel_flags((n, n, n))
    sim = LBM((n, n, n), 0.55, (1e-6, 0, 0), "f32", flags=flags, steps_per_pass=2)
    rng = np.random.default_rng(10232)
    zyx = [(n - 1, n - 2, n - 1), (n - 1, 1, 0), (n - 2, n - 2, n - 2), (0, 1, 0), (127, 13, 63),
           (128, 14, 64), (1022, 1021, 1022), (896, 1015, 960)]
    zyx += [(int(z), int(y), int(x)) for z, y, x in
            zip(rng.integers(0, n, 40), rng.integers(1, n - 1, 40), rng.integers(0, n, 40))]
    _sampled_two_steps(sim, flags, [(z * n + y) * n + x for z, y, x in zyx], 0.55, (1e-6, 0, 0))
    del sim
    torch.cuda.empty_cache()


@pytest.mark.parametrize("spp", [0, 2])
@pytest.mark.parametrize("case", ["porous", "moving_walls", "incompressible", "periodic_ragged"])
def test_step2_from_stores_both_states(case, spp):
    """lbm_step2_from (the adjoint's recomputation): mid == one step_from,
    dst == two, bit for bit, on arbitrary grids; the context's own grids and
    time are untouched.  spp = 2: a context made for pairs, whose resting
    walls go through the link mask."""
    shape = (21, 17, 70) if case == "periodic_ragged" else (12, 15, 66)
    say("step2_from", case, shape)
    kw = dict(u0=_u0(shape, 11))
    if case in ("porous", "incompressible"):
        kw["flags"] = I.random_flags(shape, 12, solid_fraction=0.2, noforce_fraction=0.1)
    elif case == "moving_walls":
        kw["flags"] = (I.random_flags(shape, 13, solid_fraction=0.1, noforce_fraction=0.1)
                       | I.cavity_flags(shape))
        kw["wall_u"] = (0.03, 0.01, -0.02)
    if "flags" in kw:
        kw["u0"][:, torch.from_numpy(kw["flags"] & 1 == 1)] = 0
    eq = "incompressible" if case == "incompressible" else "qian"
    sim = LBM(shape, 0.62, (3e-5, -1e-5, 2e-5), "f32", equilibrium=eq, steps_per_pass=spp,
              **kw).step(3)
    src = sim.grids[sim.current].clone()
    t0, cur0 = sim.t, sim.current
    a1, a2, m, d = (sim.new_grid() for _ in range(4))
    for g_ in (a1, a2, m, d):
        g_.fill_(7)  # the padding stays as it was: compare the written cells only
    sim.step_from(src, a1)
    sim.step_from(a1, a2)
    sim.step2_from(src, m, d)
    torch.cuda.synchronize()
    assert sim.t == t0 and sim.current == cur0
    assert torch.equal(sim.grids[sim.current], src)
    assert torch.equal(m, a1) and torch.equal(d, a2)


def test_step2_from_rejects_other_storage():
    sim = LBM((8, 8, 64), 0.7, (0, 0, 0), "f16", f16_scale_log2=10)
    a, b, c = sim.new_grid(), sim.new_grid(), sim.new_grid()
    with pytest.raises(A.LBMError) as e:
        sim.step2_from(a, b, c)
    assert e.value.status == A.LBM_E_UNSUPPORTED
    sim32 = LBM((8, 8, 64), 0.7, (0, 0, 0), "f32")
    a = sim32.new_grid()
    with pytest.raises(A.LBMError) as e:
        sim32.step2_from(a, a, sim32.new_grid())
    assert e.value.status == A.LBM_E_ARG


@pytest.mark.parametrize("storage,n", [("f32", 48), ("f32", 160), ("f16", 160), ("f64", 96)])
def test_automatic_steps_per_pass(storage, n):
    """steps_per_pass = "auto" (LBM_STEPS_AUTO): fused pairs where the pass
    fills the GPU, single steps on small grids -- the same bits as single
    steps either way (48^3 falls back; 160^3 and the FP64 96^3 fuse)."""
    shape = (n, n, n)
    say("automatic steps per pass", storage, shape)
    flags = I.random_flags(shape, 17, solid_fraction=0.1, noforce_fraction=0.05)
    u0 = _u0(shape, 18)
    u0[:, torch.from_numpy(flags & 1 == 1)] = 0
    s = 10 if storage == "f16" else 0
    kw = dict(flags=flags, u0=u0, f16_scale_log2=s)
    one = LBM(shape, 0.6, (1e-5, 0, 0), storage, **kw).step(7)
    auto = LBM(shape, 0.6, (1e-5, 0, 0), storage, steps_per_pass="auto", **kw).step(7)
    torch.cuda.synchronize()
    assert _same(one, auto)

"""Python front-end of the gfx950 D3Q19 BGK library.

PyTorch provides device memory and the stream; every step of the solver --
initialisation, the fused stream-collide update, macroscopic fields, FP64
reductions, and the adjoint -- runs in the HIP kernels behind the C ABI of
include/lbm.h.  Shapes are (nz, ny, nx); fields are [nz, ny, nx] and
[3, nz, ny, nx]; populations [19, nz, ny, x_stride] in the interface order.
"""
import ctypes
import math

import torch

from . import _abi as A

STORAGE = {"f32": A.LBM_F32, "f16": A.LBM_F16, "bf16": A.LBM_BF16, "f64": A.LBM_F64,
           "f32x": A.LBM_F32X}
EQUILIBRIUM = {"qian": A.LBM_EQ_QIAN, "incompressible": A.LBM_EQ_INCOMPRESSIBLE}
TORCH_DTYPE = {A.LBM_F32: torch.float32, A.LBM_F16: torch.float16,
               A.LBM_BF16: torch.bfloat16, A.LBM_F64: torch.float64, A.LBM_F32X: torch.float32}


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _aligned(t, what):
    if t.data_ptr() % 256:
        raise ValueError(f"{what} must be 256-byte aligned")
    return t


def _as_field(x, shape, dtype, device, what):
    """A contiguous device tensor of the given shape and dtype (a copy when
    the caller's tensor differs); None stays None."""
    if x is None:
        return None
    t = torch.as_tensor(x)
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.to(device=device, dtype=dtype).contiguous()


class LBM:
    """One D3Q19 BGK simulation on a periodic box (walls and obstacles are
    solid flag bits).  ``storage`` in {'f32', 'f16', 'bf16', 'f64', 'f32x'}
    ('f32x': FP32 storage with FP64 collision arithmetic).  ``wall_u``: the
    velocity of the cells flagged solid + moving (bit 2); ``equilibrium``:
    'qian' (u = j/rho) or 'incompressible' (He-Luo, u = j/rho0);
    ``obstacle_kernel=1`` selects the split design (a separate bounce-back
    kernel before each step) instead of the fused solid markers;
    ``steps_per_pass=2`` runs pairs of steps as one temporally blocked pass
    (same results, bit for bit); ``steps_per_pass="auto"`` does so where the
    pass fills the GPU (from about 128^3 cells on) and runs single steps
    elsewhere."""

    def __init__(self, shape, tau, force=(0.0, 0.0, 0.0), storage="f32", flags=None, u0=None,
                 rho0=None, f16_scale_log2=0, x_align=0, device="cuda", wall_u=(0.0, 0.0, 0.0),
                 equilibrium="qian", obstacle_kernel=0, steps_per_pass=0):
        self.shape = tuple(int(s) for s in shape)
        if len(self.shape) != 3:
            raise ValueError("shape must be (nz, ny, nx)")
        self.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        self.dtype = TORCH_DTYPE[self.storage]
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the solver runs on a GPU device")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.tau = float(tau)
        self.force = tuple(float(f) for f in force)
        self.wall_u = tuple(float(v) for v in wall_u)
        self.equilibrium = EQUILIBRIUM[equilibrium] if isinstance(equilibrium, str) \
            else int(equilibrium)
        self.params = A.params(self.shape, tau, self.force, self.storage, f16_scale_log2, x_align,
                               self.wall_u, self.equilibrium, obstacle_kernel, steps_per_pass)
        xs, ds, gb, sb, ab = A.lbm_query(self.params)
        self.x_stride, self.dir_stride = xs, ds
        self.grid_bytes, self.adj_partials_bytes = gb, ab
        nz, ny, nx = self.shape
        self.flags = _as_field(flags, self.shape, torch.uint8, self.device, "flags")
        self.rho0 = _as_field(rho0, self.shape, torch.float32, self.device, "rho0")
        self.u0 = _as_field(u0, (3,) + self.shape, torch.float32, self.device, "u0")
        self.grids = [_aligned(torch.empty(gb, dtype=torch.uint8, device=self.device), "grid")
                      for _ in range(2)]
        self.scratch = _aligned(torch.empty(sb, dtype=torch.uint8, device=self.device), "scratch")
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = A.lbm_init(self.params, _ptr(self.grids[0]), _ptr(self.grids[1]),
                              _ptr(self.flags), _ptr(self.scratch), _ptr(self.rho0),
                              _ptr(self.u0), ctypes.c_void_p(self.stream.cuda_stream))

    # -- state --------------------------------------------------------------
    @property
    def t(self):
        return A.lbm_time(self.ctx)

    @property
    def current(self):
        return A.lbm_current(self.ctx)

    def grid_view(self, buf, dtype=None):
        """A grid-layout buffer viewed as [19, nz, ny, x_stride] (the direction
        arrays dir_stride elements apart): a raw byte buffer in the storage
        dtype (or `dtype`), or a typed buffer (e.g. an FP32 adjoint grid) as is."""
        nz, ny, _ = self.shape
        t = buf.view(dtype or self.dtype) if buf.dtype == torch.uint8 else buf
        xs = self.x_stride
        return torch.as_strided(t, (19, nz, ny, xs), (self.dir_stride, ny * xs, xs, 1))

    def populations(self):
        """View of the current grid: offsets g = f* - w (FP16: 2^s g)."""
        return self.grid_view(self.grids[self.current])

    def new_grid(self):
        return _aligned(torch.empty(self.grid_bytes, dtype=torch.uint8, device=self.device), "grid")

    # -- the hot path -------------------------------------------------------
    def step(self, n=1):
        A.lbm_step(self.ctx, n)
        return self

    def step_from(self, src, dst):
        A.lbm_step_from(self.ctx, _ptr(_aligned(src, "src")), _ptr(_aligned(dst, "dst")))

    def step2_from(self, src, mid, dst):
        """Two steps from ``src`` in one fused pass: ``mid`` gets the first
        state, ``dst`` the second (FP32 storage)."""
        A.lbm_step2_from(self.ctx, _ptr(_aligned(src, "src")), _ptr(_aligned(mid, "mid")),
                         _ptr(_aligned(dst, "dst")))

    def macroscopics(self, f64=False):
        dt = torch.float64 if f64 else torch.float32
        rho = torch.empty(self.shape, dtype=dt, device=self.device)
        u = torch.empty((3,) + self.shape, dtype=dt, device=self.device)
        (A.lbm_macroscopics_f64 if f64 else A.lbm_macroscopics)(self.ctx, _ptr(rho), _ptr(u))
        return rho, u

    def reduce(self):
        """Device tensor (float64, 5): mass, momentum x/y/z, kinetic energy."""
        out = torch.empty(5, dtype=torch.float64, device=self.device)
        A.lbm_reduce(self.ctx, _ptr(out))
        return out

    # -- checkpoint / resume --------------------------------------------------
    def save(self, dst=None):
        dst = self.new_grid() if dst is None else _aligned(dst, "dst")
        A.lbm_save(self.ctx, _ptr(dst))
        return dst

    def restore(self, src, t):
        A.lbm_restore(self.ctx, _ptr(src), t)

    def refresh_solids(self):
        """Rewrite the solid-cell markers of the current grid (after
        populations were written into it directly) and the two-step pass's
        link mask (after the flags were changed in place)."""
        A.lbm_refresh_solids(self.ctx)

    def set_current(self, parity, t):
        A.lbm_set_current(self.ctx, parity, t)

    def pull_copy(self, src, dst):
        """Pull-copy probe: dst_i(x) = src_i(x - c_i) over this grid layout
        (periodic, no geometry, no collision), launched like the step."""
        A.lbm_pull_copy(self.ctx, _ptr(_aligned(src, "src")), _ptr(_aligned(dst, "dst")))
        return self

    def use_graphs(self, steps_per_graph):
        """Replay HIP graphs of `steps_per_graph` (even) captured steps in
        step() -- for launch-bound small grids; 0 turns it off."""
        A.lbm_use_graphs(self.ctx, steps_per_graph)
        return self

    def close(self):
        if getattr(self, "ctx", None):
            A.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stream_copy(dst, src, stream=None):
    """STREAM copy dst = src of whole tensors on the GPU (bandwidth probe)."""
    if dst.numel() * dst.element_size() != src.numel() * src.element_size():
        raise ValueError("size mismatch")
    s = torch.cuda.current_stream() if stream is None else stream
    A.lbm_stream_copy(_ptr(_aligned(dst, "dst")), _ptr(_aligned(src, "src")),
                      src.numel() * src.element_size(), ctypes.c_void_p(s.cuda_stream))


def copy_probe(dst, src, vec_per_thread=1, nontemporal=False, blocks=0, stream=None):
    """A variant of the copy dst = src for the bandwidth sweep (16-byte
    elements per thread, non-temporal accesses, grid-stride block count)."""
    if dst.numel() * dst.element_size() != src.numel() * src.element_size():
        raise ValueError("size mismatch")
    s = torch.cuda.current_stream() if stream is None else stream
    A.lbm_copy_probe(_ptr(_aligned(dst, "dst")), _ptr(_aligned(src, "src")),
                     src.numel() * src.element_size(), vec_per_thread, int(bool(nontemporal)),
                     blocks, ctypes.c_void_p(s.cuda_stream))


# The reverse sweep recomputes two states per fused pass (lbm_step2_from)
# from this many cells on: measured, the backward runs 3% faster at 256^3
# and 6% slower at 128^3, where the pass has too few blocks to fill the GPU.
FUSED_RECOMPUTE_MIN_CELLS = 1 << 24


class _Rollout(torch.autograd.Function):
    """(rho_T, u_T) after `steps` updates from f*(0) = f^eq(1, u0) under the
    body force g; backward runs the hand-written adjoint kernels with forward
    checkpoints every k steps and recomputation inside each segment."""

    @staticmethod
    def forward(ctx, u0, g, steps, tau, flags, k, wall_u, equilibrium, steps_per_pass):
        force = [float(v) for v in g.detach().double().cpu().tolist()]
        sim = LBM(u0.shape[1:], tau, force, "f32", flags=flags, u0=u0.detach(), device=u0.device,
                  wall_u=wall_u, equilibrium=equilibrium, steps_per_pass=steps_per_pass)
        ckpts = []
        for t in range(0, steps, k):  # a checkpoint at the start of every segment of k steps
            ckpts.append(sim.save())
            sim.step(min(k, steps - t))
        rho, u = sim.macroscopics()
        ctx.sim, ctx.ckpts, ctx.steps, ctx.k = sim, ckpts, steps, k
        ctx.g_meta = (g.dtype, g.device)
        return rho, u

    @staticmethod
    def backward(ctx, g_rho, g_u):
        """Reverse sweep in pull form: nu^T from the seed at f*(T-1), then
        nu^{m+1} from nu^{m+2} at f*(m) for m = T-2 .. 0, then dL/du0 from
        nu^1; the f*(m) are recomputed segment by segment from the
        checkpoints, latest segment first."""
        sim, ckpts, steps, k = ctx.sim, ctx.ckpts, ctx.steps, ctx.k
        dev = sim.device
        nfl = sim.grid_bytes // 4
        nu = [torch.empty(nfl, dtype=torch.float32, device=dev) for _ in range(2)]
        partials = torch.empty(sim.adj_partials_bytes // 8, dtype=torch.float64, device=dev)
        gr = None if g_rho is None else g_rho.to(torch.float32).contiguous()
        gu = None if g_u is None else g_u.to(torch.float32).contiguous()
        cur = 0
        seg = [None] + [sim.new_grid() for _ in range(min(k, steps) - 1)]
        fused = math.prod(sim.shape) >= FUSED_RECOMPUTE_MIN_CELLS
        for s in range(len(ckpts) - 1, -1, -1):
            t0, t1 = s * k, min(s * k + k, steps)
            seg[0] = ckpts[s]
            j = 1
            while j < t1 - t0:  # recompute the segment's states
                if fused and j + 1 < t1 - t0:  # two states per pass
                    sim.step2_from(seg[j - 1], seg[j], seg[j + 1])
                    j += 2
                else:
                    sim.step_from(seg[j - 1], seg[j])
                    j += 1
            for m in range(t1 - 1, t0 - 1, -1):  # f*(m) gives nu^{m+1}
                if m == steps - 1:
                    A.lbm_adjoint_seed(sim.ctx, _ptr(seg[m - t0]), _ptr(gr), _ptr(gu),
                                       _ptr(nu[cur]), _ptr(partials))
                else:
                    A.lbm_adjoint_step(sim.ctx, _ptr(seg[m - t0]), _ptr(nu[cur]),
                                       _ptr(nu[cur ^ 1]), _ptr(partials))
                    cur ^= 1
        du0 = torch.empty((3,) + sim.shape, dtype=torch.float32, device=dev)
        A.lbm_adjoint_init(sim.ctx, _ptr(nu[cur]), _ptr(sim.rho0), _ptr(sim.u0), _ptr(du0))
        dF = torch.empty(3, dtype=torch.float64, device=dev)
        A.lbm_adjoint_finish_dF(sim.ctx, _ptr(partials), _ptr(dF))
        gdt, gdev = ctx.g_meta
        return du0, dF.to(device=gdev, dtype=gdt), None, None, None, None, None, None, None


def rollout(u0, g, *, steps, tau, flags=None, checkpoint_every=20, wall_u=(0.0, 0.0, 0.0),
            equilibrium="qian", steps_per_pass=0):
    """Differentiable D3Q19 BGK rollout (FP32 storage): returns (rho_T, u_T)
    with gradients for the initial velocity ``u0`` [3, nz, ny, nx] and the
    body-force density ``g`` [3].  Moving walls and the incompressible
    equilibrium are supported (no gradient for the wall velocity).
    ``steps_per_pass=2`` runs the forward sweep in fused pairs of steps (the
    same states bit for bit, so the same gradients); the reverse sweep
    recomputes single states between checkpoints either way."""
    if u0.dim() != 4 or u0.shape[0] != 3:
        raise ValueError("u0 must be [3, nz, ny, nx]")
    if g.numel() != 3:
        raise ValueError("g must have 3 components")
    if steps < 1 or checkpoint_every < 1:
        raise ValueError("steps and checkpoint_every must be >= 1")
    return _Rollout.apply(u0, g.reshape(3), int(steps), float(tau), flags, int(checkpoint_every),
                          tuple(float(v) for v in wall_u), equilibrium, int(steps_per_pass))

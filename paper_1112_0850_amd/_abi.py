"""ctypes declarations of the C ABI in include/lbm.h.

Argument marshalling only: every step of the solver runs in the gfx950
kernels of ``liblbm.so``.  Importing this module fails loudly if the library
has not been built; there is no fallback implementation.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_E_ARG, LBM_E_HIP, LBM_E_UNSUPPORTED, LBM_E_STATE = 0, -1, -2, -3, -4
LBM_F32, LBM_F16, LBM_BF16, LBM_F64, LBM_F32X = 0, 1, 2, 3, 4
LBM_FLAG_SOLID, LBM_FLAG_NOFORCE, LBM_FLAG_MOVING = 1, 2, 4
LBM_EQ_QIAN, LBM_EQ_INCOMPRESSIBLE = 0, 1
LBM_STEPS_AUTO = -1

STATUS_NAMES = {0: "LBM_OK", -1: "LBM_E_ARG", -2: "LBM_E_HIP", -3: "LBM_E_UNSUPPORTED",
                -4: "LBM_E_STATE"}


class lbm_params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("storage", C.c_int32), ("f16_scale_log2", C.c_int32), ("x_align", C.c_int32),
                ("tau", C.c_double), ("force", C.c_double * 3), ("wall_u", C.c_double * 3),
                ("equilibrium", C.c_int32), ("obstacle_kernel", C.c_int32),
                ("steps_per_pass", C.c_int32)]


class LBMError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_vp = C.c_void_p
_st = C.c_int32
_SIGNATURES = {
    "lbm_query": (_st, [C.POINTER(lbm_params), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                        C.POINTER(C.c_size_t),
                        C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "lbm_bytes_per_update": (C.c_int32, [C.c_int32]),
    "lbm_lattice": (None, [C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "lbm_solid_markers": (_st, [C.c_int32, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "lbm_init": (_st, [C.POINTER(_vp), C.POINTER(lbm_params), _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "lbm_step": (_st, [_vp, C.c_int32]),
    "lbm_step_from": (_st, [_vp, _vp, _vp]),
    "lbm_step2_from": (_st, [_vp, _vp, _vp, _vp]),
    "lbm_macroscopics": (_st, [_vp, _vp, _vp]),
    "lbm_macroscopics_f64": (_st, [_vp, _vp, _vp]),
    "lbm_reduce": (_st, [_vp, _vp]),
    "lbm_reduce_noalloc": (_st, [_vp, _vp]),
    "lbm_current": (C.c_int32, [_vp]),
    "lbm_time": (C.c_int64, [_vp]),
    "lbm_set_current": (_st, [_vp, C.c_int32, C.c_int64]),
    "lbm_set_stream": (_st, [_vp, _vp]),
    "lbm_refresh_solids": (_st, [_vp]),
    "lbm_save": (_st, [_vp, _vp]),
    "lbm_restore": (_st, [_vp, _vp, C.c_int64]),
    "lbm_adjoint_seed": (_st, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "lbm_adjoint_step": (_st, [_vp, _vp, _vp, _vp, _vp]),
    "lbm_adjoint_init": (_st, [_vp, _vp, _vp, _vp, _vp]),
    "lbm_adjoint_finish_dF": (_st, [_vp, _vp, _vp]),
    "lbm_stream_copy": (_st, [_vp, _vp, C.c_size_t, _vp]),
    "lbm_copy_probe": (_st, [_vp, _vp, C.c_size_t, C.c_int32, C.c_int32, C.c_int32, _vp]),
    "lbm_pull_copy": (_st, [_vp, _vp, _vp]),
    "lbm_use_graphs": (_st, [_vp, C.c_int32]),
    "lbm_destroy": (None, [_vp]),
    "lbm_last_error": (C.c_char_p, []),
}

_lib = None


def lib():
    """The loaded library (raises if it was never built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -m paper_1112_0850_amd.build); there is no CPU fallback")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status != LBM_OK:
        raise LBMError(status, lib().lbm_last_error().decode())
    return status


def params(shape, tau, force=(0.0, 0.0, 0.0), storage=LBM_F32, f16_scale_log2=0, x_align=0,
           wall_u=(0.0, 0.0, 0.0), equilibrium=LBM_EQ_QIAN, obstacle_kernel=0, steps_per_pass=0):
    nz, ny, nx = shape
    p = lbm_params()
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    p.storage = int(storage)
    p.f16_scale_log2 = int(f16_scale_log2)
    p.x_align = int(x_align)
    p.tau = float(tau)
    for d in range(3):
        p.force[d] = float(force[d])
        p.wall_u[d] = float(wall_u[d])
    p.equilibrium = int(equilibrium)
    p.obstacle_kernel = int(obstacle_kernel)
    p.steps_per_pass = LBM_STEPS_AUTO if steps_per_pass == "auto" else int(steps_per_pass)
    return p


# -- thin wrappers with the C names ----------------------------------------

def lbm_query(p):
    """(x_stride, dir_stride, grid_bytes, scratch_bytes, adj_partials_bytes)."""
    xs, ds = C.c_int64(), C.c_int64()
    gb, sb, ab = C.c_size_t(), C.c_size_t(), C.c_size_t()
    check(lib().lbm_query(C.byref(p), C.byref(xs), C.byref(ds), C.byref(gb), C.byref(sb),
                          C.byref(ab)))
    return xs.value, ds.value, gb.value, sb.value, ab.value


def lbm_bytes_per_update(storage):
    return int(lib().lbm_bytes_per_update(int(storage)))


def lbm_lattice():
    e = (C.c_int32 * 57)()
    w = (C.c_double * 19)()
    opp = (C.c_int32 * 19)()
    lib().lbm_lattice(e, w, opp)
    return [tuple(e[3 * i:3 * i + 3]) for i in range(19)], list(w), list(opp)


def lbm_solid_markers(storage):
    """(resting, moving-wall) marker bits of a storage type."""
    r, m = C.c_uint64(), C.c_uint64()
    check(lib().lbm_solid_markers(int(storage), C.byref(r), C.byref(m)))
    return r.value, m.value


def lbm_init(p, grid_a, grid_b, flags, scratch, rho0, u0, stream):
    ctx = _vp()
    check(lib().lbm_init(C.byref(ctx), C.byref(p), grid_a, grid_b, flags, scratch, rho0, u0,
                         stream))
    return ctx


def lbm_step(ctx, n):
    check(lib().lbm_step(ctx, int(n)))


def lbm_step_from(ctx, src, dst):
    check(lib().lbm_step_from(ctx, src, dst))


def lbm_step2_from(ctx, src, mid, dst):
    check(lib().lbm_step2_from(ctx, src, mid, dst))


def lbm_macroscopics(ctx, rho, u):
    check(lib().lbm_macroscopics(ctx, rho, u))


def lbm_macroscopics_f64(ctx, rho, u):
    check(lib().lbm_macroscopics_f64(ctx, rho, u))


def lbm_reduce(ctx, out5):
    check(lib().lbm_reduce(ctx, out5))


def lbm_reduce_noalloc(ctx, out5):
    check(lib().lbm_reduce_noalloc(ctx, out5))


def lbm_current(ctx):
    return int(lib().lbm_current(ctx))


def lbm_time(ctx):
    return int(lib().lbm_time(ctx))


def lbm_set_current(ctx, parity, t):
    check(lib().lbm_set_current(ctx, int(parity), int(t)))


def lbm_set_stream(ctx, stream):
    check(lib().lbm_set_stream(ctx, stream))


def lbm_refresh_solids(ctx):
    check(lib().lbm_refresh_solids(ctx))


def lbm_save(ctx, dst):
    check(lib().lbm_save(ctx, dst))


def lbm_restore(ctx, src, t):
    check(lib().lbm_restore(ctx, src, int(t)))


def lbm_adjoint_seed(ctx, fstar_prev, dL_drho, dL_du, nu_T, partials):
    check(lib().lbm_adjoint_seed(ctx, fstar_prev, dL_drho, dL_du, nu_T, partials))


def lbm_adjoint_step(ctx, fstar_prev, nu_np1, nu_n, partials):
    check(lib().lbm_adjoint_step(ctx, fstar_prev, nu_np1, nu_n, partials))


def lbm_adjoint_init(ctx, nu_1, rho0, u0, dL_du0):
    check(lib().lbm_adjoint_init(ctx, nu_1, rho0, u0, dL_du0))


def lbm_adjoint_finish_dF(ctx, partials, dLdF3):
    check(lib().lbm_adjoint_finish_dF(ctx, partials, dLdF3))


def lbm_stream_copy(dst, src, n_bytes, stream):
    check(lib().lbm_stream_copy(dst, src, int(n_bytes), stream))


def lbm_copy_probe(dst, src, n_bytes, vec_per_thread, nontemporal, blocks, stream):
    check(lib().lbm_copy_probe(dst, src, int(n_bytes), int(vec_per_thread), int(nontemporal),
                               int(blocks), stream))


def lbm_pull_copy(ctx, src, dst):
    check(lib().lbm_pull_copy(ctx, src, dst))


def lbm_use_graphs(ctx, steps_per_graph):
    check(lib().lbm_use_graphs(ctx, int(steps_per_graph)))


def lbm_destroy(ctx):
    lib().lbm_destroy(ctx)


def lbm_last_error():
    return lib().lbm_last_error().decode()

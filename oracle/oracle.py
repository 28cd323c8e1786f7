"""numpy front-end of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
import this module.  It marshals numpy arrays into ``liboracle.so`` (built
from ``lbm_oracle.c`` by ``oracle/build.py``); it imports nothing from the
GPU package and the GPU package imports nothing from here.

Array conventions (all float64, C-contiguous):
  populations f[19, nz, ny, nx] in interface direction order,
  scalar fields [nz, ny, nx], vector fields [3, nz, ny, nx],
  flags uint8[nz, ny, nx] (bit0 solid, bit1 no body force, bit2 moving
  wall) or None.
Model options taken by the grid functions: ``wall_u`` (velocity of the solid
cells with the moving-wall bit, or None) and ``incompressible`` (False: the
Qian equilibrium with u = j/rho; True: the He-Luo equilibrium, u = j/rho0).
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

Q = 19
_lib = None


def load(path):
    """Load an oracle shared library and declare its C signatures."""
    L = C.CDLL(path)
    dp = C.POINTER(C.c_double)
    u8p = C.POINTER(C.c_uint8)
    ip = C.POINTER(C.c_int)
    i, d, l = C.c_int, C.c_double, C.c_long
    sig = {
        "oracle_lattice": [ip, dp, ip],
        "oracle_equilibrium": [d, dp, i, dp],
        "oracle_guo_source": [d, dp, dp, dp],
        "oracle_collide": [d, dp, i, dp, dp],
        "oracle_collide_jacobian": [d, dp, i, dp, dp, dp],
        "oracle_init": [i, i, i, u8p, i, dp, dp, dp],
        "oracle_step": [i, i, i, d, dp, u8p, dp, i, dp, l],
        "oracle_stream": [i, i, i, u8p, dp, dp, l],
        "oracle_macroscopics": [i, i, i, dp, u8p, i, dp, dp, dp],
        "oracle_reduce": [i, i, i, dp, u8p, i, dp, dp],
        "oracle_adjoint_seed": [i, i, i, dp, u8p, i, dp, dp, dp, dp, dp],
        "oracle_adjoint_step": [i, i, i, d, dp, u8p, dp, i, dp, dp, dp, dp],
        "oracle_adjoint_init": [i, i, i, u8p, i, dp, dp, dp, dp, dp],
        "oracle_adjoint_collide": [i, i, i, d, dp, u8p, i, dp, dp, dp, dp],
        "oracle_stream_transpose": [i, i, i, u8p, dp, dp],
        "oracle_host_copy": [dp, dp, l, i],
        "oracle_threads": [],
        "oracle_set_threads": [i],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_double if name == "oracle_host_copy" else C.c_int
    return L


def lib():
    """The oracle library: ``liboracle.so``, or the build named by the
    ORACLE_LIB environment variable (the sanitizer build of the tests)."""
    global _lib
    if _lib is None:
        _lib = load(os.environ.get("ORACLE_LIB") or _build.ensure_built())
    return _lib


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _u8(a):
    if a is None:
        return None
    assert a.dtype == np.uint8 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_uint8))


def _vec3(v):
    return np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(3))


def _wall(wall_u):
    return None if wall_u is None else _d(_vec3(wall_u))


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def _flags(flags, shape):
    if flags is None:
        return None
    f = np.ascontiguousarray(flags, dtype=np.uint8)
    assert f.shape == tuple(shape)
    return f


# -- lattice and single-cell functions ------------------------------------

def lattice():
    """(e int[19,3], w float64[19], opp int[19]) in interface order."""
    e = np.zeros((Q, 3), dtype=np.int32)
    w = np.zeros(Q)
    opp = np.zeros(Q, dtype=np.int32)
    _check(lib().oracle_lattice(e.ctypes.data_as(C.POINTER(C.c_int)), _d(w),
                                opp.ctypes.data_as(C.POINTER(C.c_int))), "lattice")
    return e, w, opp


def equilibrium(rho, u, incompressible=False):
    out = np.zeros(Q)
    _check(lib().oracle_equilibrium(float(rho), _d(_vec3(u)), int(incompressible), _d(out)),
           "equilibrium")
    return out


def guo_source(omega, u, F):
    out = np.zeros(Q)
    _check(lib().oracle_guo_source(float(omega), _d(_vec3(u)), _d(_vec3(F)), _d(out)), "guo")
    return out


def collide(tau, F, f, incompressible=False):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(Q)
    _check(lib().oracle_collide(float(tau), _d(_vec3(F)), int(incompressible), _d(f), _d(out)),
           "collide")
    return out


def collide_jacobian(tau, F, f, incompressible=False):
    f = np.ascontiguousarray(f, dtype=np.float64)
    J = np.zeros((Q, Q))
    JF = np.zeros((Q, 3))
    _check(lib().oracle_collide_jacobian(float(tau), _d(_vec3(F)), int(incompressible), _d(f),
                                         _d(J), _d(JF)), "jacobian")
    return J, JF


# -- grid functions --------------------------------------------------------

def init(shape, flags=None, rho0=None, u0=None, incompressible=False):
    """f*(0) = f^eq(rho0, u0) for a grid of shape (nz, ny, nx)."""
    nz, ny, nx = shape
    fl = _flags(flags, shape)
    r = None if rho0 is None else np.ascontiguousarray(rho0, dtype=np.float64)
    u = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64)
    f = np.zeros((Q, nz, ny, nx))
    _check(lib().oracle_init(nx, ny, nz, _u8(fl), int(incompressible), _d(r), _d(u), _d(f)),
           "init")
    return f


def step(f, tau, F=(0.0, 0.0, 0.0), flags=None, n=1, wall_u=None, incompressible=False):
    """n stream-collide steps; returns a new array."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    _, nz, ny, nx = f.shape
    fl = _flags(flags, (nz, ny, nx))
    _check(lib().oracle_step(nx, ny, nz, float(tau), _d(_vec3(F)), _u8(fl), _wall(wall_u),
                             int(incompressible), _d(f), int(n)), "step")
    return f


def stream(f, flags=None, n=1, wall_u=None):
    """n pure streaming steps (with bounce-back); returns a new array."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    _, nz, ny, nx = f.shape
    fl = _flags(flags, (nz, ny, nx))
    _check(lib().oracle_stream(nx, ny, nz, _u8(fl), _wall(wall_u), _d(f), int(n)), "stream")
    return f


def macroscopics(f, F=(0.0, 0.0, 0.0), flags=None, incompressible=False):
    f = np.ascontiguousarray(f, dtype=np.float64)
    _, nz, ny, nx = f.shape
    fl = _flags(flags, (nz, ny, nx))
    rho = np.zeros((nz, ny, nx))
    u = np.zeros((3, nz, ny, nx))
    _check(lib().oracle_macroscopics(nx, ny, nz, _d(_vec3(F)), _u8(fl), int(incompressible),
                                     _d(f), _d(rho), _d(u)), "macroscopics")
    return rho, u


def reduce(f, F=(0.0, 0.0, 0.0), flags=None, incompressible=False):
    """{M, Px, Py, Pz, E} over fluid cells, FP64."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    _, nz, ny, nx = f.shape
    fl = _flags(flags, (nz, ny, nx))
    out = np.zeros(5)
    _check(lib().oracle_reduce(nx, ny, nz, _d(_vec3(F)), _u8(fl), int(incompressible), _d(f),
                               _d(out)), "reduce")
    return out


def adjoint_seed(fT, dL_drho, dL_du, F=(0.0, 0.0, 0.0), flags=None, incompressible=False):
    """(lambda^T, dL/dF contribution) from dL/drho_T and dL/du_T."""
    fT = np.ascontiguousarray(fT, dtype=np.float64)
    _, nz, ny, nx = fT.shape
    fl = _flags(flags, (nz, ny, nx))
    gr = None if dL_drho is None else np.ascontiguousarray(dL_drho, dtype=np.float64)
    gu = None if dL_du is None else np.ascontiguousarray(dL_du, dtype=np.float64)
    lam = np.zeros_like(fT)
    dF = np.zeros(3)
    _check(lib().oracle_adjoint_seed(nx, ny, nz, _d(_vec3(F)), _u8(fl), int(incompressible),
                                     _d(fT), _d(gr), _d(gu), _d(lam), _d(dF)), "adjoint_seed")
    return lam, dF


def adjoint_step(fn, lam_np1, tau, F=(0.0, 0.0, 0.0), flags=None, wall_u=None,
                 incompressible=False):
    """(lambda^n, dL/dF contribution of this step) from f*(n) and lambda^{n+1}."""
    fn = np.ascontiguousarray(fn, dtype=np.float64)
    lam_np1 = np.ascontiguousarray(lam_np1, dtype=np.float64)
    _, nz, ny, nx = fn.shape
    fl = _flags(flags, (nz, ny, nx))
    lam = np.zeros_like(fn)
    dF = np.zeros(3)
    _check(lib().oracle_adjoint_step(nx, ny, nz, float(tau), _d(_vec3(F)), _u8(fl),
                                     _wall(wall_u), int(incompressible), _d(fn), _d(lam_np1),
                                     _d(lam), _d(dF)), "adjoint_step")
    return lam, dF


def adjoint_collide(f_pre, lam, tau, F=(0.0, 0.0, 0.0), flags=None, incompressible=False):
    """(mu = J(f_pre)^T lam, dL/dF contribution JF(f_pre)^T lam): the collision's
    part of a reverse step at a pre-collision state f_pre."""
    f_pre = np.ascontiguousarray(f_pre, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    _, nz, ny, nx = f_pre.shape
    fl = _flags(flags, (nz, ny, nx))
    mu = np.zeros_like(f_pre)
    dF = np.zeros(3)
    _check(lib().oracle_adjoint_collide(nx, ny, nz, float(tau), _d(_vec3(F)), _u8(fl),
                                        int(incompressible), _d(f_pre), _d(lam), _d(mu), _d(dF)),
           "adjoint_collide")
    return mu, dF


def stream_transpose(mu, flags=None):
    """lam = stream^T(mu): the transposed streaming with bounce-back (a gather)."""
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    _, nz, ny, nx = mu.shape
    fl = _flags(flags, (nz, ny, nx))
    lam = np.zeros_like(mu)
    _check(lib().oracle_stream_transpose(nx, ny, nz, _u8(fl), _d(mu), _d(lam)), "stream_transpose")
    return lam


def adjoint_init(lam0, u0, flags=None, rho0=None, incompressible=False):
    """(dL/du0, dL/drho0) from lambda^0."""
    lam0 = np.ascontiguousarray(lam0, dtype=np.float64)
    _, nz, ny, nx = lam0.shape
    fl = _flags(flags, (nz, ny, nx))
    u = np.ascontiguousarray(u0, dtype=np.float64)
    r = None if rho0 is None else np.ascontiguousarray(rho0, dtype=np.float64)
    gu = np.zeros((3, nz, ny, nx))
    gr = np.zeros((nz, ny, nx))
    _check(lib().oracle_adjoint_init(nx, ny, nz, _u8(fl), int(incompressible), _d(r), _d(u),
                                     _d(lam0), _d(gu), _d(gr)), "adjoint_init")
    return gu, gr


def threads():
    return int(lib().oracle_threads())


def set_threads(n):
    """Thread count of the following oracle calls; returns the count in use."""
    return int(lib().oracle_set_threads(int(n)))


def host_copy_gbs(n=1 << 25, reps=5):
    """Host STREAM-copy bandwidth in GB/s (read + write bytes, no write-allocate)."""
    import time
    a = np.ones(n)
    c = np.zeros(n)
    lib().oracle_host_copy(_d(c), _d(a), n, 1)
    t0 = time.perf_counter()
    lib().oracle_host_copy(_d(c), _d(a), n, reps)
    dt = time.perf_counter() - t0
    return 2 * 8 * n * reps / dt / 1e9

"""Pins of the oracle's discrete adjoint (no GPU): the per-cell Jacobian
against central differences of the collision, an exact dot-product test of
the transposed streaming with bounce-back, and the full reverse sweep against
FP64 central differences of the whole rollout."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1112_0850_amd import inputs as I
from tests import lattice_ref as R


@pytest.mark.parametrize("inc", [False, True])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_collision_jacobian_vs_central_differences(seed, inc):
    _, w, _ = R.e_w_opp()
    rng = np.random.default_rng(seed)
    f = w * (1 + 0.1 * rng.standard_normal(19))
    tau = 0.55 + 0.5 * rng.random()
    F = 1e-2 * rng.standard_normal(3)
    J, JF = O.collide_jacobian(tau, F, f, incompressible=inc)
    col = lambda F_, f_: O.collide(tau, F_, f_, incompressible=inc)
    h = 1e-6
    Jfd = np.zeros((19, 19))
    for j in range(19):
        d = np.zeros(19)
        d[j] = h
        Jfd[:, j] = (col(F, f + d) - col(F, f - d)) / (2 * h)
    JFfd = np.zeros((19, 3))
    for a in range(3):
        d = np.zeros(3)
        d[a] = h
        JFfd[:, a] = (col(F + d, f) - col(F - d, f)) / (2 * h)
    assert np.abs(J - Jfd).max() < 1e-9 * np.abs(J).max()
    assert np.abs(JF - JFfd).max() < 1e-9 * np.abs(JF).max()


def test_transposed_streaming_dot_product_exact():
    """<P x, y> == <x, P^T y> for pull + bounce-back (tau = inf, F = 0 makes
    the collision Jacobian the identity); integer data make it exact."""
    shape = (5, 4, 6)
    flags = I.random_flags(shape, 3, solid_fraction=0.25)
    rng = np.random.default_rng(8)
    x = rng.integers(-50, 50, size=(19,) + shape).astype(np.float64)
    y = rng.integers(-50, 50, size=(19,) + shape).astype(np.float64)
    x[:, flags == 1] = 0
    y[:, flags == 1] = 0
    Px = O.stream(x, flags, n=1)
    # f*(n) only enters through the collision Jacobian, which is I here;
    # any valid state works.
    _, w, _ = R.e_w_opp()
    fn = np.broadcast_to(w[:, None, None, None], x.shape).copy()
    fn[:, flags == 1] = 0
    PTy, dF = O.adjoint_step(fn, y, np.inf, (0, 0, 0), flags)
    assert (Px * y).sum() == (x * PTy).sum()
    assert not PTy[:, flags == 1].any()


def test_stream_transpose_dot_product_exact():
    """The exported transposed streaming: <P x, y> == <x, P^T y> exactly for
    the streaming P of the forward oracle (integer data), and the adjoint
    step is P^T after the collision part at the streamed state, bit for bit."""
    shape = (4, 5, 7)
    flags = I.random_flags(shape, 9, solid_fraction=0.3)
    rng = np.random.default_rng(10)
    x = rng.integers(-50, 50, size=(19,) + shape).astype(np.float64)
    y = rng.integers(-50, 50, size=(19,) + shape).astype(np.float64)
    x[:, flags == 1] = 0
    y[:, flags == 1] = 0
    PTy = O.stream_transpose(y, flags)
    assert (O.stream(x, flags, n=1) * y).sum() == (x * PTy).sum()
    assert not PTy[:, flags == 1].any()
    tau, F = 0.7, (1e-3, -2e-3, 5e-4)
    fn = O.step(O.init(shape, flags, None, 0.03 * (rng.random((3,) + shape) - 0.5)), tau, F, flags)
    lam = rng.standard_normal((19,) + shape)
    lam[:, flags == 1] = 0
    mu, dF1 = O.adjoint_collide(O.stream(fn, flags), lam, tau, F, flags)
    lam_n, dF2 = O.adjoint_step(fn, lam, tau, F, flags)
    assert np.array_equal(O.stream_transpose(mu, flags), lam_n) and np.array_equal(dF1, dF2)


def test_adjoint_collide_vs_central_differences():
    """sum lam . (Omega(f + e v) - Omega(f - e v)) / 2e == sum v . mu on a
    grid of cells (Omega applied cell by cell through oracle.collide), and
    the same for a force perturbation against dL/dF."""
    shape = (2, 3, 4)
    _, w, _ = R.e_w_opp()
    rng = np.random.default_rng(21)
    flags = np.zeros(shape, np.uint8)
    flags[0, 1, 2] = 2  # one no-force cell
    f = w[:, None, None, None] * (1 + 0.1 * rng.standard_normal((19,) + shape))
    lam = rng.standard_normal((19,) + shape)
    v = rng.standard_normal((19,) + shape)
    tau, F = 0.66, np.array([1e-2, -2e-2, 5e-3])
    mu, dF = O.adjoint_collide(f, lam, tau, F, flags)

    def omega(ff, FF):
        out = np.zeros_like(ff)
        for z, y_, x in np.ndindex(shape):
            Fc = FF if flags[z, y_, x] != 2 else np.zeros(3)
            out[:, z, y_, x] = O.collide(tau, Fc, ff[:, z, y_, x])
        return out

    h = 1e-6
    fd = ((omega(f + h * v, F) - omega(f - h * v, F)) * lam).sum() / (2 * h)
    assert abs(fd - (v * mu).sum()) <= 1e-8 * abs(fd)
    for a in range(3):
        d = np.zeros(3)
        d[a] = h
        fdF = ((omega(f, F + d) - omega(f, F - d)) * lam).sum() / (2 * h)
        assert abs(fdF - dF[a]) <= 1e-8 * abs(fdF)


def rollout_loss(u0, F, flags, tau, steps, target, wall_u=None, inc=False):
    """L = mean over fluid cells and components of (u_T - u*)^2."""
    shape = u0.shape[1:]
    f = O.init(shape, flags, None, u0, incompressible=inc)
    f = O.step(f, tau, F, flags, n=steps, wall_u=wall_u, incompressible=inc)
    _, u = O.macroscopics(f, F, flags, incompressible=inc)
    fl = np.ones(shape, bool) if flags is None else (flags & 1) == 0
    return ((u - target) ** 2)[:, fl].mean()


def rollout_grad(u0, F, flags, tau, steps, target, wall_u=None, inc=False):
    shape = u0.shape[1:]
    fl = np.ones(shape, bool) if flags is None else (flags & 1) == 0
    states = [O.init(shape, flags, None, u0, incompressible=inc)]
    for _ in range(steps):
        states.append(O.step(states[-1], tau, F, flags, n=1, wall_u=wall_u, incompressible=inc))
    _, uT = O.macroscopics(states[-1], F, flags, incompressible=inc)
    gu = np.zeros_like(uT)
    gu[:, fl] = 2 * (uT - target)[:, fl] / (3 * fl.sum())
    lam, dF = O.adjoint_seed(states[-1], None, gu, F, flags, incompressible=inc)
    for n in range(steps - 1, -1, -1):
        lam, d = O.adjoint_step(states[n], lam, tau, F, flags, wall_u=wall_u, incompressible=inc)
        dF += d
    du0, _ = O.adjoint_init(lam, u0, flags, incompressible=inc)
    return du0, dF


@pytest.mark.parametrize("solids,walls,inc", [(False, False, False), (True, False, False),
                                              (True, True, False), (True, True, True),
                                              (False, False, True)])
def test_full_adjoint_vs_central_differences(solids, walls, inc):
    """Variants: periodic; random solids with no-force cells; moving walls
    (a lid-driven box whose lid moves along x, plus random solids) with the
    Qian or the incompressible equilibrium; periodic incompressible."""
    n, tau, steps = 8, 0.6, 25
    shape = (n, n, n)
    flags, wall_u = None, None
    if solids:
        flags = I.random_flags(shape, 31, solid_fraction=0.15, noforce_fraction=0.2)
    if walls:
        flags = flags | I.cavity_flags(shape)
        wall_u = (0.03, 0.0, 0.01)
    u0 = I.smooth_field(n, 2024, amplitude=0.02, modes=4)
    target = I.smooth_field(n, 7, amplitude=0.02, modes=4)
    F = np.array([1e-4, -5e-5, 2e-5])
    if flags is not None:
        u0[:, flags & 1 == 1] = 0
    du0, dF = rollout_grad(u0, F, flags, tau, steps, target, wall_u, inc)
    # central differences at eps and eps/2, Richardson-extrapolated so the
    # O(eps^2) truncation cancels (the remaining error is O(eps^4)).
    def fd(fun, eps):
        d1 = (fun(eps) - fun(-eps)) / (2 * eps)
        d2 = (fun(eps / 2) - fun(-eps / 2)) / eps
        return (4 * d2 - d1) / 3

    for k, s in enumerate([101, 102]):
        v = I.smooth_field(n, s, amplitude=1.0, modes=4)
        ref = fd(lambda e: rollout_loss(u0 + e * v, F, flags, tau, steps, target, wall_u, inc),
                 1e-4)
        ad = (du0 * v).sum()
        assert abs(ad - ref) <= 1e-8 * abs(ref), (k, ad, ref)
    for a in range(3):
        d = np.zeros(3)
        d[a] = 1.0
        ref = fd(lambda e: rollout_loss(u0, F + e * d, flags, tau, steps, target, wall_u, inc),
                 1e-5)
        assert abs(dF[a] - ref) <= 1e-8 * abs(ref), (a, dF[a], ref)

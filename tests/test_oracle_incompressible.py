"""Pins of the oracle's incompressible equilibrium (He & Luo 1997; the
paper calls its solver incompressible, abstract and Sec. 2) against exact
mathematics (no GPU).  With rho0 = 1 the equilibrium is
f^eq_i = w_i [rho + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u] and u = j + F/2: its
moments, conservation by the collision, the macroscopic read-back, fixed
points, and -- because its linearisation about rest is that of the Qian
equilibrium and unidirectional flows keep rho = 1 -- the Taylor-Green
eigen-decay and the exact discrete steady Poiseuille profile."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1112_0850_amd import inputs as I
from tests import lattice_ref as R
from tests import test_oracle_dynamics as TD


@pytest.mark.parametrize("rho,u", [(1.0, (0.0, 0.0, 0.0)), (1.03, (0.05, -0.02, 0.01)),
                                   (0.97, (-0.1, 0.07, 0.03))])
def test_equilibrium_moments(rho, u):
    """sum f^eq = rho, sum f^eq c = u (rho0 u), sum f^eq c_a c_b = rho d_ab/3 + u_a u_b."""
    e, w, _ = R.e_w_opp()
    feq = O.equilibrium(rho, u, incompressible=True)
    u = np.array(u)
    assert abs(feq.sum() - rho) < 1e-15
    assert np.abs(e.T @ feq - u).max() < 1e-15
    P = np.einsum("i,ia,ib->ab", feq, e, e)
    assert np.abs(P - (rho * np.eye(3) / 3 + np.outer(u, u))).max() < 1e-15
    # the two equilibria differ by (rho - 1) times the velocity polynomial
    cu = e @ u
    diff = O.equilibrium(rho, u) - feq
    assert np.abs(diff - (rho - 1) * w * (3 * cu + 4.5 * cu * cu - 1.5 * u @ u)).max() < 1e-16


def test_collision_conserves_and_relaxes():
    e, w, _ = R.e_w_opp()
    rng = np.random.default_rng(6)
    f = w * (1 + 0.05 * rng.standard_normal(19))
    tau = 0.7
    F = np.array([1e-4, 2e-4, -1e-4])
    fs = O.collide(tau, F, f, incompressible=True)
    assert abs(fs.sum() - f.sum()) < 1e-15
    assert np.abs(e.T @ fs - (e.T @ f + F)).max() < 1e-15
    fs0 = O.collide(tau, np.zeros(3), f, incompressible=True)
    feq = O.equilibrium(f.sum(), e.T @ f, incompressible=True)
    Pneq = np.einsum("i,ia,ib->ab", f - feq, e, e)
    Pneq_s = np.einsum("i,ia,ib->ab", fs0 - feq, e, e)
    assert np.abs(Pneq_s - (1 - 1 / tau) * Pneq).max() < 1e-15


def test_macroscopics_read_back_the_initial_state():
    shape = (4, 5, 6)
    flags = I.random_flags(shape, 9, solid_fraction=0.2)
    rho0 = 1 + 0.02 * I.random_offsets(shape, 1)[0] / 1e-2
    u0 = 0.04 * I.random_offsets(shape, 2)[:3] / 1e-2
    f = O.init(shape, flags, rho0, u0, incompressible=True)
    rho, u = O.macroscopics(f, (0, 0, 0), flags, incompressible=True)
    fl = flags & 1 == 0
    assert np.abs(rho - rho0)[fl].max() < 1e-15
    assert np.abs(u - u0)[:, fl].max() < 1e-16


def test_uniform_equilibrium_stays_fixed():
    shape = (4, 5, 6)
    u0 = np.zeros((3,) + shape)
    u0[0], u0[1], u0[2] = 0.05, -0.03, 0.02
    rho0 = np.full(shape, 1.04)
    f0 = O.init(shape, None, rho0, u0, incompressible=True)
    f = O.step(f0, 0.7, (0, 0, 0), None, n=20, incompressible=True)
    assert np.abs(f - f0).max() < 1e-13


def test_taylor_green_decay():
    n, tau = 32, 0.8
    shape = (n, n, n)
    u0 = I.taylor_green(shape, 0.01)
    f = O.init(shape, None, None, u0, incompressible=True)
    ts, amps = [], []
    for t in range(0, 201, 10):
        if t:
            f = O.step(f, tau, n=10, incompressible=True)
        _, u = O.macroscopics(f, incompressible=True)
        ts.append(t)
        amps.append((u * u0).sum() / (u0 * u0).sum())
    ts, amps = np.array(ts), np.array(amps)
    m = ts >= 20
    rate = -np.polyfit(ts[m], np.log(amps[m]), 1)[0]
    k = np.array([2 * math.pi / n, 2 * math.pi / n, 0.0])
    nu = (tau - 0.5) / 3
    assert abs(rate - nu * (k @ k)) < 0.01 * nu * (k @ k)
    eig = TD._shear_eigen_rate(tau, k)
    assert abs(rate - eig) < 1e-4 * eig


@pytest.mark.parametrize("tau", [0.6, 1.0])
def test_poiseuille_exact_steady_state(tau):
    ny, F = 32, 1e-6
    shape = (1, ny, 1)
    fl = I.channel_flags(shape)
    nu = (tau - 0.5) / 3
    H = ny - 2
    steps = int(1.2 * 12 * H * H / (nu * math.pi ** 2) * math.log(10))
    f = O.step(O.init(shape, fl, incompressible=True), tau, (F, 0, 0), fl, n=steps,
               incompressible=True)
    rho, u = O.macroscopics(f, (F, 0, 0), fl, incompressible=True)
    ua = TD._poiseuille_exact(ny, tau, F)[1:-1]
    assert np.abs(u[0, 0, 1:-1, 0] - ua).max() <= 1e-10 * ua.max()
    assert np.abs(rho[0, 1:-1, 0] - 1).max() < 1e-10


def test_reduction_uses_reference_density():
    """Momentum and energy of the incompressible model are rho0 u and
    rho0 |u|^2 / 2 with rho0 = 1."""
    shape = (3, 4, 5)
    rho0 = 1 + 0.03 * I.random_offsets(shape, 5)[0] / 1e-2
    u0 = 0.04 * I.random_offsets(shape, 6)[:3] / 1e-2
    f = O.init(shape, None, rho0, u0, incompressible=True)
    r = O.reduce(f, (0, 0, 0), None, incompressible=True)
    assert abs(r[0] - rho0.sum()) < 1e-12
    assert np.abs(r[1:4] - u0.reshape(3, -1).sum(1)).max() < 1e-14
    assert abs(r[4] - 0.5 * (u0 * u0).sum()) < 1e-14

"""Pins of the oracle's full update against closed forms and invariants:
fixed points, conservation, Taylor-Green decay (continuum and the exact
eigenvalue of the linearised one-step operator) and the exact discrete
steady Poiseuille profile of BGK + half-way bounce-back + Guo forcing."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1112_0850_amd import inputs as I
from tests import lattice_ref as R


def test_uniform_equilibrium_stays_fixed():
    shape = (4, 5, 6)
    u0 = np.zeros((3,) + shape)
    u0[0], u0[1], u0[2] = 0.05, -0.03, 0.02
    f0 = O.init(shape, None, None, u0)
    f = O.step(f0, 0.7, (0, 0, 0), None, n=20)
    assert np.abs(f - f0).max() < 1e-13


def test_rest_state_with_solids_stays_fixed():
    shape = (5, 6, 7)
    flags = I.random_flags(shape, 11, solid_fraction=0.3)
    f0 = O.init(shape, flags)
    f = O.step(f0, 0.55, (0, 0, 0), flags, n=10)
    assert np.abs(f - f0).max() < 1e-15


@pytest.mark.parametrize("with_solids", [False, True])
def test_conservation(with_solids):
    """Periodic box: mass is constant; without solids momentum grows by
    N_fluid F per step; with bounce-back walls mass is still constant."""
    shape = (8, 7, 6)
    flags = I.random_flags(shape, 21, solid_fraction=0.2) if with_solids else None
    F = np.array([1e-5, -2e-5, 3e-6])
    u0 = 0.02 * I.random_offsets(shape, 4)[:3] / 1e-2
    f = O.init(shape, flags, None, u0)
    r0 = O.reduce(f, F, flags)
    n = 50
    f = O.step(f, 0.8, F, flags, n=n)
    r1 = O.reduce(f, F, flags)
    assert abs(r1[0] - r0[0]) <= 1e-12 * r0[0]
    if not with_solids:
        nfl = np.prod(shape)
        assert np.abs(r1[1:4] - r0[1:4] - n * nfl * F).max() <= 1e-12 * nfl * np.abs(F).max() * n


def _shear_eigen_rate(tau, k):
    """-ln|lambda| of the transverse shear mode of M(k) = [I - w(I - E)] S(k),
    E_ij = w_i (1 + 3 c_i.c_j), S = diag(exp(-i k.c_j)) (linearised one-step
    operator about rest, pull streaming)."""
    e, w, _ = R.e_w_opp()
    e = e.astype(float)
    om = 1.0 / tau
    E = w[:, None] * (1 + 3 * e @ e.T)
    M = (np.eye(19) - om * (np.eye(19) - E)) @ np.diag(np.exp(-1j * (e @ k)))
    lam, V = np.linalg.eig(M)
    t = np.cross(k, [0.0, 0.0, 1.0])
    t /= np.linalg.norm(t)
    best = None
    for j in range(19):
        mom = e.T @ V[:, j]
        if abs(t @ mom) > 0.1 * np.linalg.norm(mom) and abs(lam[j].imag) < 1e-12:
            if best is None or abs(lam[j]) > abs(lam[best]):
                best = j
    return -math.log(abs(lam[best]))


def test_taylor_green_decay():
    """32^3 periodic, tau = 0.8, u0 = 0.01: the amplitude decays at the
    linear shear eigenvalue (to 1e-4) and at nu |k|^2, nu = (tau - 1/2)/3
    (to 1%), fitted on t in [20, 200]."""
    n, tau = 32, 0.8
    shape = (n, n, n)
    u0 = I.taylor_green(shape, 0.01)
    f = O.init(shape, None, None, u0)
    ts, amps = [], []
    for t in range(0, 201, 10):
        if t:
            f = O.step(f, tau, n=10)
        _, u = O.macroscopics(f)
        ts.append(t)
        amps.append((u * u0).sum() / (u0 * u0).sum())
    ts, amps = np.array(ts), np.array(amps)
    m = ts >= 20
    rate = -np.polyfit(ts[m], np.log(amps[m]), 1)[0]
    k = np.array([2 * math.pi / n, 2 * math.pi / n, 0.0])
    nu = (tau - 0.5) / 3
    assert abs(rate - nu * (k @ k)) < 0.01 * nu * (k @ k)
    eig = _shear_eigen_rate(tau, k)
    assert abs(rate - eig) < 1e-4 * eig


def _poiseuille_exact(ny, tau, F):
    """Steady x-velocity of BGK + half-way bounce-back + Guo forcing between
    walls at y_a = 1/2 and y_b = ny - 3/2:
    u(y) = F/(2 nu) (y - y_a)(y_b - y) + F (16 Lambda - 3)/(24 nu),
    Lambda = (tau - 1/2)^2; the slip term vanishes at Lambda = 3/16."""
    nu = (tau - 0.5) / 3
    y = np.arange(ny, dtype=np.float64)
    ya, yb = 0.5, ny - 1.5
    lam = (tau - 0.5) ** 2
    return F / (2 * nu) * (y - ya) * (yb - y) + F * (16 * lam - 3) / (24 * nu)


@pytest.mark.parametrize("tau", [0.6, 0.5 + math.sqrt(3) / 4, 1.0])
def test_poiseuille_exact_steady_state(tau):
    ny, F = 32, 1e-6
    shape = (1, ny, 1)
    fl = I.channel_flags(shape)
    f = O.init(shape, fl)
    nu = (tau - 0.5) / 3
    H = ny - 2
    steps = int(1.2 * 12 * H * H / (nu * math.pi ** 2) * math.log(10))
    f = O.step(f, tau, (F, 0, 0), fl, n=steps)
    rho, u = O.macroscopics(f, (F, 0, 0), fl)
    ua = _poiseuille_exact(ny, tau, F)[1:-1]
    assert np.abs(u[0, 0, 1:-1, 0] - ua).max() <= 1e-10 * ua.max()
    assert np.abs(u[1:, 0, 1:-1, 0]).max() <= 1e-10 * ua.max()
    assert np.abs(rho[0, 1:-1, 0] - 1).max() < 1e-10


def test_poiseuille_startup_transient():
    """Start-up flow from rest: u = u_steady - sum_{n odd} 4 F H^2/(nu pi^3 n^3)
    sin(n pi eta / H) exp(-n^2 pi^2 nu t / H^2), within 1% of max u."""
    ny, F, tau, t = 32, 1e-6, 0.6, 5000
    H = ny - 2
    nu = (tau - 0.5) / 3
    shape = (1, ny, 1)
    fl = I.channel_flags(shape)
    f = O.step(O.init(shape, fl), tau, (F, 0, 0), fl, n=t)
    _, u = O.macroscopics(f, (F, 0, 0), fl)
    eta = np.arange(ny) - 0.5
    ref = _poiseuille_exact(ny, tau, F)
    for n in range(1, 400, 2):
        ref -= 4 * F * H * H / (nu * math.pi ** 3 * n ** 3) * np.sin(n * math.pi * eta / H) * \
            math.exp(-n * n * math.pi ** 2 * nu * t / H ** 2)
    ux = u[0, 0, 1:-1, 0]
    assert np.abs(ux - ref[1:-1]).max() < 0.01 * ux.max()

"""Pins of the oracle's lattice and single-cell physics against exact
mathematics (no GPU).  Lattice: D3Q19 (Sec. 2, Qian et al. 1992); moment
identities of the equilibrium and of the Guo forcing term."""
from fractions import Fraction
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from tests import lattice_ref as R


def test_enumeration_has_19_velocities():
    assert len(R.enumerated()) == 19
    assert sorted(R.enumerated()) == sorted(R.INTERFACE_ORDER)


def test_oracle_lattice_matches_interface_table():
    e, w, opp = O.lattice()
    e_r, w_r, opp_r = R.e_w_opp()
    assert np.array_equal(e, e_r)
    assert np.array_equal(w, w_r)  # exact: 1/3, 1/18, 1/36 round identically
    assert np.array_equal(opp, opp_r)
    assert np.array_equal(e[opp], -e)


def test_isotropy_exact_rationals():
    """sum w = 1; sum w c = 0; sum w c_a c_b = d_ab/3; odd 3rd moment = 0;
    sum w c_a c_b c_c c_d = (d_ab d_cd + d_ac d_bd + d_ad d_bc)/9."""
    cs = R.INTERFACE_ORDER
    ws = [R.WEIGHT_BY_NORM2[sum(x * x for x in c)] for c in cs]
    assert sum(ws) == 1
    d = lambda a, b: 1 if a == b else 0
    for a in range(3):
        assert sum(w * c[a] for w, c in zip(ws, cs)) == 0
        for b in range(3):
            assert sum(w * c[a] * c[b] for w, c in zip(ws, cs)) == Fraction(d(a, b), 3)
            for g in range(3):
                assert sum(w * c[a] * c[b] * c[g] for w, c in zip(ws, cs)) == 0
                for h in range(3):
                    lhs = sum(w * c[a] * c[b] * c[g] * c[h] for w, c in zip(ws, cs))
                    rhs = Fraction(d(a, b) * d(g, h) + d(a, g) * d(b, h) + d(a, h) * d(b, g), 9)
                    assert lhs == rhs


@pytest.mark.parametrize("rho,u", [(1.0, (0.0, 0.0, 0.0)), (1.03, (0.05, -0.02, 0.01)),
                                   (0.97, (-0.1, 0.07, 0.03))])
def test_equilibrium_moments(rho, u):
    """sum f^eq = rho, sum f^eq c = rho u, sum f^eq c_a c_b = rho (u_a u_b + d_ab/3)."""
    e, w, _ = R.e_w_opp()
    feq = O.equilibrium(rho, u)
    u = np.array(u)
    assert abs(feq.sum() - rho) < 1e-15
    assert np.abs(e.T @ feq - rho * u).max() < 1e-15
    P = np.einsum("i,ia,ib->ab", feq, e, e)
    assert np.abs(P - rho * (np.outer(u, u) + np.eye(3) / 3)).max() < 1e-15
    # closed form at rest: f^eq = rho w
    if not u.any():
        assert np.abs(feq - rho * w).max() < 1e-16


@pytest.mark.parametrize("omega", [1 / 0.55, 1 / 0.8, 1.0])
def test_guo_moments(omega):
    """sum S = 0 and sum S c = (1 - omega/2) F (Guo et al. 2002)."""
    e, w, _ = R.e_w_opp()
    u = np.array([0.03, -0.01, 0.02])
    F = np.array([1e-3, -2e-3, 5e-4])
    S = O.guo_source(omega, u, F)
    assert abs(S.sum()) < 1e-18
    assert np.abs(e.T @ S - (1 - omega / 2) * F).max() < 1e-18
    # second moment: (1 - omega/2)(u F + F u) (Guo's design condition)
    P = np.einsum("i,ia,ib->ab", S, e, e)
    assert np.abs(P - (1 - omega / 2) * (np.outer(u, F) + np.outer(F, u))).max() < 1e-18


def test_collision_conserves_and_relaxes():
    """Collision keeps mass; momentum gains F; the non-equilibrium part of
    the second moment relaxes by (1 - omega) at F = 0."""
    e, w, _ = R.e_w_opp()
    rng = np.random.default_rng(5)
    f = w * (1 + 0.05 * rng.standard_normal(19))
    tau = 0.7
    F = np.array([1e-4, 2e-4, -1e-4])
    fs = O.collide(tau, F, f)
    assert abs(fs.sum() - f.sum()) < 1e-15
    assert np.abs(e.T @ fs - (e.T @ f + F)).max() < 1e-15
    fs0 = O.collide(tau, np.zeros(3), f)
    rho = f.sum()
    u = e.T @ f / rho
    feq = O.equilibrium(rho, u)
    Pneq = np.einsum("i,ia,ib->ab", f - feq, e, e)
    Pneq_s = np.einsum("i,ia,ib->ab", fs0 - feq, e, e)
    assert np.abs(Pneq_s - (1 - 1 / tau) * Pneq).max() < 1e-15


def test_rest_state_is_fixed():
    _, w, _ = R.e_w_opp()
    fs = O.collide(0.6, np.zeros(3), w)
    assert np.abs(fs - w).max() < 1e-15  # round-off of the FP64 sums

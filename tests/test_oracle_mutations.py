"""The oracle's pins are sensitive: each plausible mistake planted in a copy
of the oracle source (a dropped or altered term, a wrong sign, a wrong index)
is caught by at least one pin.  Runs on the CPU only; the planted copies are
compiled into a temporary directory and never used elsewhere."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import oracle as O
from tests import test_oracle_adjoint as TA
from tests import test_oracle_dynamics as TD
from tests import test_oracle_incompressible as TI
from tests import test_oracle_lattice as TL
from tests import test_oracle_streaming as TS
from tests import test_oracle_switches as TSW
from tests import test_oracle_walls as TW

SRC = os.path.join(os.path.dirname(O.__file__), "lbm_oracle.c")


def _eq():
    TL.test_equilibrium_moments(1.03, (0.05, -0.02, 0.01))


def _guo():
    TL.test_guo_moments(1 / 0.8)


def _collide():
    TL.test_collision_conserves_and_relaxes()


def _stream():
    TS.test_bounce_back_streaming_brute_force((4, 5, 6), 3)


def _poiseuille():
    TD.test_poiseuille_exact_steady_state(0.6)


def _tgv():
    TD.test_taylor_green_decay()


def _jac():
    TA.test_collision_jacobian_vs_central_differences(0, False)


def _dot():
    TA.test_transposed_streaming_dot_product_exact()


def _full_adj():
    TA.test_full_adjoint_vs_central_differences(True, False, False)


def _conservation():
    TD.test_conservation(False)


def _momentum():
    TW.test_momentum_one_streaming_step((0.07, 0.0, 0.0))


def _couette():
    TW.test_couette_exact_steady_state(1.0, False)


def _inc_eq():
    TI.test_equilibrium_moments(1.03, (0.05, -0.02, 0.01))


def _inc_collide():
    TI.test_collision_conserves_and_relaxes()


def _inc_read_back():
    TI.test_macroscopics_read_back_the_initial_state()


def _inc_jac():
    TA.test_collision_jacobian_vs_central_differences(1, True)


def _inc_full_adj():
    TA.test_full_adjoint_vs_central_differences(False, False, True)


def _walls_full_adj():
    TA.test_full_adjoint_vs_central_differences(True, True, False)


def _adj_collide_fd():
    TA.test_adjoint_collide_vs_central_differences()


def _transpose_dot():
    TA.test_stream_transpose_dot_product_exact()


def _noforce_gain():
    TSW.test_noforce_switch_momentum_gain(1)


def _noforce_rest():
    TSW.test_noforce_switch_one_step_from_rest()


def _qian_reduce():
    TSW.test_qian_reduction_of_an_equilibrium_state()


def _drho0():
    TSW.test_initial_density_gradient_vs_central_differences()


# (planted change: old text -> new text, first occurrence only; pins that must fail)
MUTATIONS = {
    "equilibrium_second_order": ("double poly = 3.0 * cu + 4.5 * cu * cu", "double poly = 3.0 * cu + 4.0 * cu * cu",
                                 [_eq, _tgv]),
    "equilibrium_uu_term": ("double poly = 3.0 * cu + 4.5 * cu * cu - 1.5 * uu;",
                            "double poly = 3.0 * cu + 4.5 * cu * cu - 0.5 * uu;",
                            [_eq]),
    "guo_prefactor_sign": ("S[i] = (1.0 - 0.5 * omega)", "S[i] = (1.0 + 0.5 * omega)", [_guo]),
    "guo_dropped_u_term": ("(3.0 * (cF - uF) + 9.0 * cu * cF)", "(3.0 * cF + 9.0 * cu * cF)",
                           [_guo, _poiseuille]),
    "half_force_in_velocity": ("u[d] = (j[d] + 0.5 * F[d]) / (incomp", "u[d] = (j[d]) / (incomp",
                               [_poiseuille, _collide]),
    "relaxation_sign": ("fout[i] = f[i] - omega * (f[i] - feq[i])",
                        "fout[i] = f[i] + omega * (f[i] - feq[i])", [_collide, _tgv]),
    "bounce_back_not_reversed": ("dst[c * Q + OPP[i]] = src[c * Q + i];",
                                 "dst[c * Q + i] = src[c * Q + i];", [_stream, _poiseuille]),
    "macroscopic_force_shift": ("(m[d] - 0.5 * Fc[d]) / (incomp", "(m[d] + 0.5 * Fc[d]) / (incomp",
                                [_poiseuille]),
    "weight_of_diagonals": ("(n2 == 1) ? 1.0 / 18.0 : 1.0 / 36.0", "(n2 == 1) ? 1.0 / 18.0 : 1.0 / 37.0",
                            [_eq, _conservation]),
    "jacobian_velocity_derivative": (": (C[jj][a] - u[a]) / rho;", ": (C[jj][a] + u[a]) / rho;",
                                     [_jac]),
    "jacobian_force_half": ("(omega * dfeq_du[a] + dS_du[a]) / (2.0 * rho_u);",
                            "(omega * dfeq_du[a] + dS_du[a]) / rho_u;", [_jac]),
    "adjoint_transpose_index": ("mu[t * Q + i] : mu[c * Q + OPP[i]]", "mu[t * Q + i] : mu[c * Q + i]",
                                [_dot]),
    "adjoint_seed_force_sign": ("acc[d] += -gu[d] / (2.0 * rho_u);", "acc[d] += gu[d] / (2.0 * rho_u);",
                                [_full_adj]),
    "adjoint_init_dropped_term": ("9.0 * cu * C[i][a] - 3.0 * u[a]);\n      }\n    }\n    for (int a = 0; a < 3; ++a) dL_du0",
                                  "9.0 * cu * C[i][a]);\n      }\n    }\n    for (int a = 0; a < 3; ++a) dL_du0",
                                  [_full_adj]),
    "moving_wall_sign": ("src[c * Q + i] - 6.0 * W[i] * cdot(i, wall_u)",
                         "src[c * Q + i] + 6.0 * W[i] * cdot(i, wall_u)", [_momentum, _couette]),
    "moving_wall_factor": ("src[c * Q + i] - 6.0 * W[i] * cdot(i, wall_u)",
                           "src[c * Q + i] - 3.0 * W[i] * cdot(i, wall_u)", [_momentum, _couette]),
    "moving_wall_direction": ("src[c * Q + i] - 6.0 * W[i] * cdot(i, wall_u)",
                              "src[c * Q + i] - 6.0 * W[i] * cdot(OPP[i], wall_u)",
                              [_momentum, _couette]),
    "moving_bit_ignored": ("else if (wall_u && is_moving(flags, t))",
                           "else if (wall_u && 0 && is_moving(flags, t))",
                           [_momentum, _couette]),
    "adjoint_recompute_without_walls": ("stream_push(&g, flags, wall_u, a, b);\n    rc = adjoint_collide_aos",
                                        "stream_push(&g, flags, NULL, a, b);\n    rc = adjoint_collide_aos",
                                        [_walls_full_adj]),
    "adjoint_collide_transposed": ("s += lam[c * Q + i] * J[i][jj];", "s += lam[c * Q + i] * J[jj][i];",
                                   [_adj_collide_fd, _full_adj]),
    "stream_transpose_without_bounce": ("v = !is_solid(flags, t) ? mu[t * Q + i] : mu[c * Q + OPP[i]];",
                                        "v = mu[t * Q + i];", [_dot, _transpose_dot]),
    "incompressible_equilibrium_rho": ("incomp ? W[i] * (rho + poly)", "incomp ? W[i] * rho * (1.0 + poly)",
                                       [_inc_eq]),
    "incompressible_velocity": ("(j[d] + 0.5 * F[d]) / (incomp ? 1.0 : rho)", "(j[d] + 0.5 * F[d]) / rho",
                                [_inc_collide]),
    "incompressible_macroscopics": ("(m[d] - 0.5 * Fc[d]) / (incomp ? 1.0 : r)",
                                    "(m[d] - 0.5 * Fc[d]) / r", [_inc_read_back]),
    "incompressible_jacobian_du": ("double du_df = incomp ? C[jj][a] :",
                                   "double du_df = incomp ? (C[jj][a] - u[a]) :", [_inc_jac]),
    "incompressible_jacobian_drho": ("double dfeq_drho = incomp ? W[i] :",
                                     "double dfeq_drho = incomp ? W[i] * (1.0 + poly) :", [_inc_jac]),
    "noforce_ignored": ("int off = flags && (flags[c] & FLAG_NOFORCE);", "int off = 0;",
                        [_noforce_gain, _noforce_rest]),
    "noforce_inverted": ("int off = flags && (flags[c] & FLAG_NOFORCE);",
                         "int off = !(flags && (flags[c] & FLAG_NOFORCE));",
                         [_noforce_gain, _noforce_rest]),
    "macroscopics_noforce_ignored": ("    double Fc[3];\n    cell_force(flags, c, F, Fc);\n    if (rho) rho[c] = r;",
                                     "    double Fc[3] = {F[0], F[1], F[2]};\n    if (rho) rho[c] = r;",
                                     [_noforce_rest]),
    "qian_energy_without_rho": ("s[4] += 0.5 * m * dot3(uc, uc);", "s[4] += 0.5 * dot3(uc, uc);",
                                [_qian_reduce]),
    "qian_momentum_without_rho": ("s[1 + d] += m * uc[d];", "s[1 + d] += uc[d];", [_qian_reduce]),
    "adjoint_init_drho_dropped_uu": ("4.5 * cu * cu - 1.5 * uu));", "4.5 * cu * cu));", [_drho0]),
    "adjoint_init_drho_dropped_cu": ("W[i] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu));",
                                     "W[i] * (1.0 + 4.5 * cu * cu - 1.5 * uu));", [_drho0]),
    "incompressible_seed": ("v += gu[d] * (incomp ? ABI_E[k][d] :",
                            "v += gu[d] * (incomp ? ABI_E[k][d] - uc[d] :", [_inc_full_adj]),
}


@pytest.fixture(scope="module")
def workdir():
    with tempfile.TemporaryDirectory() as d:
        yield d


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, workdir):
    old, new, checks = MUTATIONS[name]
    src = open(SRC).read()
    assert old in src, f"mutation anchor for {name} not found"
    mutated = src.replace(old, new, 1)
    cpath = os.path.join(workdir, f"{name}.c")
    lpath = os.path.join(workdir, f"lib{name}.so")
    open(cpath, "w").write(mutated)
    subprocess.run(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-o", lpath, cpath, "-lm"], check=True)
    saved = O._lib
    O._lib = O.load(lpath)
    try:
        caught = []
        for chk in checks:
            try:
                chk()
                caught.append(False)
            except AssertionError:
                caught.append(True)
        assert any(caught), f"no pin caught the planted mistake {name}"
        # every listed pin is expected to catch it
        assert all(caught), f"{name}: caught by {[c.__name__ for c, k in zip(checks, caught) if k]}"
    finally:
        O._lib = saved


def test_unmutated_oracle_passes_the_same_checks():
    for chk in {c for _, _, cs in MUTATIONS.values() for c in cs}:
        chk()

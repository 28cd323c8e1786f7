"""Host-side pin of the collision coefficients compiled into the kernels:
rounded next to the exact D3Q19 values (w, 3w, 9w/2, 9w) and chosen so the
conservation identities hold exactly on the rounded values (sum W = 1,
2 a_axis + 8 a_diag = 1, 2 c_axis + 8 c_diag = 3/2, 2 q_axis + 8 q_diag = 3),
for both compute precisions.  Reads the constants from the source."""
import os
import re
from fractions import Fraction as Fr

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = open(os.path.join(ROOT, "paper_1112_0850_amd", "csrc", "d3q19.h")).read()


def _consts(tname):
    block = re.search(r"struct Coef<%s> \{(.*?)\};" % tname, SRC, re.S).group(1)
    vals = dict(re.findall(r"(W0|W1|W2|A1|A2) = (0x[0-9a-fA-F.]+p[+-]?\d+)", block))
    return {k: Fr(float.fromhex(v)) for k, v in vals.items()}


@pytest.mark.parametrize("tname,dt,tol", [("float", np.float32, 2e-7), ("double", np.float64, 1e-15)])
def test_coefficients(tname, dt, tol):
    c = _consts(tname)
    assert set(c) == {"W0", "W1", "W2", "A1", "A2"}
    for k, v in c.items():  # representable in the compute type
        assert Fr(float(dt(float(v)))) == v, k
    assert c["W0"] + 6 * c["W1"] + 12 * c["W2"] == 1
    assert 2 * c["A1"] + 8 * c["A2"] == 1
    exact = {"W0": Fr(1, 3), "W1": Fr(1, 18), "W2": Fr(1, 36), "A1": Fr(1, 6), "A2": Fr(1, 12)}
    for k in exact:
        assert abs(float(c[k] / exact[k]) - 1) < tol, k
    # the exact binary coefficients 9w/2 and 9w
    assert 2 * Fr(1, 4) + 8 * Fr(1, 8) == Fr(3, 2)
    assert 2 * Fr(1, 2) + 8 * Fr(1, 4) == 3
    assert "C(0.25) : C(0.125)" in SRC and "C(0.5) : C(0.25)" in SRC

"""An independent, test-side description of the D3Q19 lattice.

Used only to pin the oracle and the library's exported tables: velocities are
enumerated here from the definition (every c in {-1,0,1}^3 with |c|^2 <= 2),
and the interface order is the table documented in include/lbm.h, retyped.
"""
import itertools
from fractions import Fraction

import numpy as np

INTERFACE_ORDER = [
    (0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
    (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1),
    (1, 0, -1), (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1),
]
WEIGHT_BY_NORM2 = {0: Fraction(1, 3), 1: Fraction(1, 18), 2: Fraction(1, 36)}


def enumerated():
    return [c for c in itertools.product((-1, 0, 1), repeat=3) if sum(x * x for x in c) <= 2]


def e_w_opp():
    e = np.array(INTERFACE_ORDER, dtype=np.int64)
    w = np.array([float(WEIGHT_BY_NORM2[int(c @ c)]) for c in e])
    opp = np.array([INTERFACE_ORDER.index(tuple(-c)) for c in e])
    return e, w, opp

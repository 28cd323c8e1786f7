"""Pins of the oracle's streaming step (Sec. 2 step 3 and the bounce-back of
the obstacle paragraph) and of its grid-level state handling (no GPU)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1112_0850_amd import inputs as I
from tests import lattice_ref as R


@pytest.mark.parametrize("shape", [(3, 4, 5), (1, 1, 1), (2, 3, 1), (5, 2, 7)])
@pytest.mark.parametrize("nsteps", [1, 3])
def test_free_streaming_is_a_cyclic_shift(shape, nsteps):
    """No solids: after n steps population i is its field shifted by n c_i."""
    e, _, _ = R.e_w_opp()
    f = I.random_offsets(shape, seed=1)
    g = O.stream(f, None, n=nsteps)
    for i in range(19):
        ref = np.roll(f[i], shift=(nsteps * e[i, 2], nsteps * e[i, 1], nsteps * e[i, 0]),
                      axis=(0, 1, 2))
        assert np.array_equal(g[i], ref)


def _brute_pull(f, flags, e, opp):
    """Half-way bounce-back as a pull, written with plain loops:
    f_i(x) = f_i(x - c_i) if that cell is fluid, else f_opp(i)(x); solid: 0."""
    nz, ny, nx = flags.shape
    out = np.zeros_like(f)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if flags[z, y, x] & 1:
                    continue
                for i in range(19):
                    sz, sy, sx = (z - e[i, 2]) % nz, (y - e[i, 1]) % ny, (x - e[i, 0]) % nx
                    if flags[sz, sy, sx] & 1:
                        out[i, z, y, x] = f[opp[i], z, y, x]
                    else:
                        out[i, z, y, x] = f[i, sz, sy, sx]
    return out


@pytest.mark.parametrize("shape,seed", [((4, 5, 6), 3), ((3, 3, 3), 4), ((2, 6, 1), 5)])
def test_bounce_back_streaming_brute_force(shape, seed):
    e, _, opp = R.e_w_opp()
    flags = I.random_flags(shape, seed, solid_fraction=0.3)
    f = I.random_offsets(shape, seed)
    f[:, flags == 1] = 0.0
    g = O.stream(f, flags, n=1)
    assert np.array_equal(g, _brute_pull(f, flags, e, opp))
    g2 = O.stream(f, flags, n=2)
    assert np.array_equal(g2, _brute_pull(_brute_pull(f, flags, e, opp), flags, e, opp))


def test_streaming_is_a_permutation_with_solids():
    """Every fluid slot value survives streaming exactly once (bijection)."""
    shape = (6, 5, 4)
    flags = I.random_flags(shape, 9, solid_fraction=0.25)
    f = np.zeros((19,) + shape)
    vals = np.arange(1, f.size + 1, dtype=np.float64).reshape(f.shape)
    f[:, flags == 0] = vals[:, flags == 0]
    g = O.stream(f, flags, n=1)
    a = np.sort(f[:, flags == 0].ravel())
    b = np.sort(g[:, flags == 0].ravel())
    assert np.array_equal(a, b)
    assert not g[:, flags == 1].any()


def test_infinite_tau_is_pure_streaming():
    """tau = +inf gives omega = 0: a full step is exactly streaming at F = 0."""
    shape = (3, 4, 5)
    flags = I.random_flags(shape, 2, solid_fraction=0.2)
    _, w, _ = R.e_w_opp()
    f = I.random_offsets(shape, 7) + w[:, None, None, None]
    f[:, flags == 1] = 0.0
    assert np.array_equal(O.step(f, np.inf, (0, 0, 0), flags, n=2), O.stream(f, flags, n=2))

"""The seeded input generators (CPU): the SplitMix64 stream against the
reference generator's published outputs for seed 0 (Steele, Lea & Flood
2014), and the stated properties of each geometry and field recipe --
seeded determinism, the sphere pack's target fraction, radii and
non-overlap under the periodic minimum image, the cavity and Couette
layouts, and the scaling of the smooth and Taylor-Green fields."""
import math

import numpy as np
import pytest

from paper_1112_0850_amd import inputs as I


def test_splitmix64_reference_outputs():
    r = I.SplitMix64(0)
    assert [r.next_u64() for _ in range(4)] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    u = I.SplitMix64(0).uniform()
    assert u == (0xE220A8397B1DCDAF >> 11) / 2.0 ** 53 and 0.0 <= u < 1.0


def _components(solid):
    """Connected solid components (6-neighbour, periodic) -> list of cell sets."""
    from scipy import ndimage
    lab, n = ndimage.label(solid)
    # merge labels that touch across the periodic faces
    parent = list(range(n + 1))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a
    for ax in range(3):
        a = np.take(lab, 0, axis=ax)
        b = np.take(lab, -1, axis=ax)
        for p, q in zip(a[(a > 0) & (b > 0)], b[(a > 0) & (b > 0)]):
            parent[find(p)] = find(q)
    roots = np.array([find(v) for v in range(n + 1)])
    return roots[lab], len(set(roots[1:]))


def test_sphere_pack_properties():
    shape = (64, 48, 56)
    f = I.sphere_pack(shape, 0.10, seed=3)
    assert f.dtype == np.uint8 and set(np.unique(f)) <= {0, I.FLAG_SOLID}
    frac = (f == I.FLAG_SOLID).mean()
    # stops at the first sphere that reaches the target: at most one sphere over
    assert 0.10 <= frac < 0.10 + (4 / 3) * math.pi * 12.5 ** 3 / np.prod(shape)
    assert np.array_equal(f, I.sphere_pack(shape, 0.10, seed=3))
    assert not np.array_equal(f, I.sphere_pack(shape, 0.10, seed=4))
    # non-overlapping spheres of radius <= 12: every solid component fits in a
    # ball of radius 12 around its centroid (periodic minimum image)
    lab, n = _components(f == I.FLAG_SOLID)
    assert n >= 5
    dims = np.array(shape)
    for c in np.unique(lab[lab > 0]):
        idx = np.argwhere(lab == c).astype(np.float64)
        ref = idx[0]
        d = idx - ref
        d -= dims * np.round(d / dims)
        pts = ref + d
        rad = np.sqrt(((pts - pts.mean(0)) ** 2).sum(1)).max()
        assert rad <= 12.5, rad


def test_sphere_pack_rejects_small_box():
    with pytest.raises(ValueError):
        I.sphere_pack((20, 64, 64), 0.1, seed=1)


def test_cavity_and_couette_layouts():
    shape = (6, 7, 8)
    c = I.cavity_flags(shape)
    S, M = I.FLAG_SOLID, I.FLAG_MOVING
    assert (c[-1] == S | M).all()
    for face in (c[0], c[:-1, 0], c[:-1, -1], c[:-1, :, 0], c[:-1, :, -1]):
        assert (face == S).all()
    assert (c[1:-1, 1:-1, 1:-1] == 0).all()
    k = I.couette_flags(shape)
    assert (k[:, 0] == S).all() and (k[:, -1] == S | M).all() and (k[:, 1:-1] == 0).all()
    ch = I.channel_flags(shape)
    assert (ch[:, 0] == S).all() and (ch[:, -1] == S).all() and (ch[:, 1:-1] == 0).all()


def test_smooth_field_scaling_and_resolution():
    u = I.smooth_field(16, 2024, amplitude=0.02, modes=4)
    assert abs(np.sqrt((u * u).sum(0)).max() - 0.02) < 1e-15
    # one seed is one continuous field: the 32^3 field sampled on every other
    # point is the 16^3 field up to the amplitude normalisation
    v = I.smooth_field(32, 2024, amplitude=0.02, modes=4)[:, ::2, ::2, ::2]
    assert abs((u * v).sum() / math.sqrt((u * u).sum() * (v * v).sum()) - 1) < 1e-12
    assert np.array_equal(u, I.smooth_field(16, 2024, amplitude=0.02, modes=4))


def test_taylor_green_field():
    u = I.taylor_green((4, 32, 32), 0.01)
    assert abs(np.abs(u[0]).max() - 0.01) < 1e-12 and not u[2].any()
    # divergence-free on the lattice's central differences to round-off
    div = (np.roll(u[0], -1, 2) - np.roll(u[0], 1, 2)) + (np.roll(u[1], -1, 1) - np.roll(u[1], 1, 1))
    assert np.abs(div).max() < 1e-15

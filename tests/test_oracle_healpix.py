"""Pins of the oracle's HEALPix directions against Gorski et al. (2005).

The ray directions of DART-Ray are HEALPix pixel centres (paper Sect. 3.1.1);
the scattered source function is sampled on HEALPix pixels too (Sect. 3.1.2).
These tests check the oracle's nested pix2vec against what the HEALPix paper
fixes: ring latitudes and longitudes in closed form, pixel counts, the
nested quad-tree (children of p are 4p..4p+3 and lie inside p, checked with an
independently written ang2pix) and the symmetry of the pixel set.
"""

import math

import numpy as np
import pytest


def ring_closed_form(nside):
    """All pixel centres (z, phi) from the ring-scheme closed forms."""
    out = []
    for i in range(1, 4 * nside):
        if i < nside:                      # north cap
            z = 1.0 - i * i / (3.0 * nside * nside)
            out += [(z, math.pi / (2 * i) * (j - 0.5)) for j in range(1, 4 * i + 1)]
        elif i <= 3 * nside:               # equatorial belt
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * nside)
            s = (i - nside + 1) % 2
            out += [(z, math.pi / (2 * nside) * (j - s / 2.0)) for j in range(1, 4 * nside + 1)]
        else:                              # south cap (mirror)
            ii = 4 * nside - i
            z = -(1.0 - ii * ii / (3.0 * nside * nside))
            out += [(z, math.pi / (2 * ii) * (j - 0.5)) for j in range(1, 4 * ii + 1)]
    return out


def ang2pix_nest(nside, v):
    """Nested pixel containing direction v (Gorski et al. 2005 construction)."""
    x, y, z = v
    phi = math.atan2(y, x)
    if phi < 0:
        phi += 2 * math.pi
    tt = (phi / (math.pi / 2)) % 4.0
    za = abs(z)
    if za <= 2.0 / 3.0:
        t1 = nside * (0.5 + tt)
        t2 = nside * z * 0.75
        jp = int(t1 - t2)
        jm = int(t1 + t2)
        ifp = jp // nside
        ifm = jm // nside
        if ifp == ifm:
            face = ifp | 4
        elif ifp < ifm:
            face = ifp
        else:
            face = ifm + 8
        ix = jm & (nside - 1)
        iy = nside - (jp & (nside - 1)) - 1
    else:
        ntt = min(3, int(tt))
        tp = tt - ntt
        tmp = nside * math.sqrt(3 * (1 - za))
        jp = min(nside - 1, int(tp * tmp))
        jm = min(nside - 1, int((1 - tp) * tmp))
        if z >= 0:
            face = ntt
            ix = nside - jm - 1
            iy = nside - jp - 1
        else:
            face = ntt + 8
            ix = jp
            iy = jm
    ipf = 0
    for b in range(30):
        ipf |= ((ix >> b) & 1) << (2 * b)
        ipf |= ((iy >> b) & 1) << (2 * b + 1)
    return face * nside * nside + ipf


@pytest.mark.parametrize("nside", [1, 2, 4, 8])
def test_pixel_centres_match_ring_closed_forms(orc, nside):
    v = orc.healpix_vecs(nside)
    assert v.shape == (12 * nside * nside, 3)
    np.testing.assert_allclose(np.linalg.norm(v, axis=1), 1.0, rtol=0, atol=1e-15)
    got = sorted((round(z, 12), round(math.atan2(y, x) % (2 * math.pi), 12)) for x, y, z in v)
    want = sorted((round(z, 12), round(p % (2 * math.pi), 12)) for z, p in ring_closed_form(nside))
    assert len(got) == len(want)
    # nested -> ring is a bijection: every closed-form centre appears exactly once
    for (zg, pg), (zw, pw) in zip(got, want):
        assert abs(zg - zw) < 1e-11
        d = abs(pg - pw)
        assert min(d, 2 * math.pi - d) < 1e-11


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 16])
def test_children_lie_inside_parent(orc, nside):
    # children of nested pixel p at 2*nside are 4p..4p+3 and their centres
    # fall inside p (checked with an independent ang2pix)
    for p in range(12 * nside * nside):
        for k in range(4):
            c = orc.healpix_vec(2 * nside, 4 * p + k)
            assert ang2pix_nest(nside, c) == p
        assert ang2pix_nest(nside, orc.healpix_vec(nside, p)) == p


def test_parent_of_fine_ray(orc):
    # a ray pixel at 8x the resolution maps to its parent by a shift of 2*3 bits
    for r in range(0, 12 * 64 * 64, 97):
        c = orc.healpix_vec(64, r)
        assert ang2pix_nest(8, c) == r >> 6


@pytest.mark.parametrize("nside", [1, 2, 4, 8])
def test_pixel_set_symmetry(orc, nside):
    v = orc.healpix_vecs(nside)
    assert np.abs(v.sum(axis=0)).max() < 1e-12
    key = {tuple(np.round(x, 10)) for x in v}
    ops = [
        lambda a: np.array([-a[1], a[0], a[2]]),   # 90 deg about z
        lambda a: np.array([a[0], a[1], -a[2]]),   # z -> -z
        lambda a: np.array([a[1], a[0], a[2]]),    # x <-> y
    ]
    for op in ops:
        img = {tuple(np.round(op(x), 10)) for x in v}
        assert img == key


def test_equal_area_and_solid_angle(orc):
    # 12 Nside^2 equal-area pixels: the j_sca array of the paper's memory
    # example has 12*4^k pixels per cell at resolution k
    for k in range(5):
        assert len(orc.healpix_vecs(2 ** k)) == 12 * 4 ** k

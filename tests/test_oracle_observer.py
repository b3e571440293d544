"""Pins of the oracle's observer maps (paper Sect. 2: the intensity reaching
an observer is I_0 e^{-tau}, summed over all cells; Sect. 3.6: internal
observers get all-sky HEALPix maps) and of its nested ang2pix.

* ang2pix against an independently written Python version and the round trip
  through pixel centres;
* a distant observer of a transparent medium receives every cell's j V: the
  image integrates to the total luminosity per steradian;
* a distant observer of a uniform absorbing slab, face-on, with image pixels
  on the cell columns: each pixel is the geometric series sum_k j V
  e^{-kappa rho (z_top - z_k)} over its column, divided by the pixel area;
* an internal observer of a transparent medium: each cell lands in the map
  pixel holding the direction to it (independent ang2pix) with j V / D^2;
* scattered light: a cell holding S in one j_sca pixel only is seen by
  observers whose direction lies in that pixel and by no other.
"""

import math

import numpy as np
import pytest

from paper_1709_03802_amd import workloads as W
from test_oracle_healpix import ang2pix_nest


@pytest.mark.parametrize("nside", [1, 2, 4, 16, 64])
def test_ang2pix_matches_independent_version_and_round_trips(orc, nside):
    rng = np.random.default_rng(nside)
    v = rng.standard_normal((2000, 3))
    for x in v:
        assert orc.healpix_pix(nside, x) == ang2pix_nest(nside, x / np.linalg.norm(x))
    for p in range(12 * nside * nside):
        assert orc.healpix_pix(nside, orc.healpix_vec(nside, p)) == p


def uniform(n, rho, emis=1.0, nz=None, size=1.0, nl=1):
    nz = n if nz is None else nz
    level, ijk = W.uniform_leaves((n, n, nz))
    N = level.shape[0]
    return W.Grid(nroot=(n, n, nz), lo=(0.0, 0.0, 0.0), root_size=size / n, level=level, ijk=ijk,
                  rho=np.full(N, float(rho)), emis=np.full((nl, N), float(emis)), kappa=np.ones(nl),
                  albedo=np.full(nl, 0.5), g=np.full(nl, 0.3), nside_sca=np.full(nl, 2, np.int32),
                  lambdas_um=np.ones(nl))


def test_distant_transparent_image_integrates_to_the_luminosity(orc):
    g = uniform(6, 0.0)
    g.emis[0] = np.random.default_rng(2).random(g.n)
    m = orc.Model(g)
    for d in ([0, 0, 1], [1, 2, 3], [-1, 0.5, 0.2]):
        ob = orc.observer("distant", dir=d, up=[0, 1, 0] if d[1] == 0 else [1, 0, 0], centre=[0.5, 0.5, 0.5],
                          pixel_size=0.05, nx=64, ny=64)
        img = m.observe(ob)
        assert img.sum() * 0.05 ** 2 == pytest.approx((g.emis[0] * g.volume()).sum(), rel=1e-12)


def test_distant_face_on_slab_is_a_geometric_series(orc):
    n, nz, kr = 4, 5, 3.0
    g = uniform(n, kr, nz=nz, size=float(n))           # unit cells, slab of 5 cells in z
    m = orc.Model(g)
    ob = orc.observer("distant", dir=[0, 0, 1], up=[0, 1, 0], centre=[n / 2, n / 2, 0.0], pixel_size=1.0,
                      nx=n, ny=n)
    img = m.observe(ob)
    # cell k of a column (centre at z = k + 1/2) is seen through nz - k - 1/2 cells of optical depth kr
    want = sum(math.exp(-kr * (nz - k - 0.5)) for k in range(nz))
    np.testing.assert_allclose(img[0], want, rtol=1e-13)


def test_internal_transparent_map_is_the_inverse_square_sum(orc):
    g = uniform(5, 0.0)
    g.emis[0] = np.random.default_rng(3).random(g.n)
    m = orc.Model(g)
    pos = np.array([0.33, 0.61, 0.47])
    nside = 8
    mp = m.observe(orc.observer("internal", pos=pos, nside_map=nside))[0]
    c = g.centres()
    own = np.all(np.abs(c - pos) <= 0.5 * g.side()[:, None], axis=1)
    want = np.zeros(12 * nside * nside)
    om = 4 * math.pi / want.size
    for i in np.flatnonzero(~own):
        v = c[i] - pos
        D2 = float(v @ v)
        want[ang2pix_nest(nside, v / math.sqrt(D2))] += g.emis[0, i] * g.volume()[i] / D2 / om
    np.testing.assert_allclose(mp, want, rtol=1e-12, atol=1e-15 * want.max())


def test_scattered_light_is_seen_only_inside_its_pixel(orc):
    g = uniform(3, 0.0, emis=0.0)
    m = orc.Model(g)
    S = np.zeros(m.s_size)
    c = 13                                            # the central cell
    p0 = 17
    m.s_block(S, 0)[c, p0] = 5.0
    v0 = orc.healpix_vec(2, p0)
    img = m.observe(orc.observer("distant", dir=v0, up=[0, 0, 1], centre=g.centres()[c], pixel_size=0.01,
                                 nx=3, ny=3), S_total=S)
    assert img.sum() * 0.01 ** 2 == pytest.approx(5.0 * 48 / (4 * math.pi), rel=1e-12)
    # a direction outside pixel 17: nothing
    v1 = orc.healpix_vec(2, 30)
    img = m.observe(orc.observer("distant", dir=v1, up=[0, 0, 1], centre=g.centres()[c], pixel_size=0.01,
                                 nx=3, ny=3), S_total=S)
    assert img.sum() == 0.0
    # in a rotated frame the pixel rotates with it
    R = W.rotation(5)
    img = m.observe(orc.observer("distant", dir=R @ v0, up=[0, 0, 1], centre=g.centres()[c], pixel_size=0.01,
                                 nx=3, ny=3, frame=R), S_total=S)
    assert img.sum() * 0.01 ** 2 == pytest.approx(5.0 * 48 / (4 * math.pi), rel=1e-12)

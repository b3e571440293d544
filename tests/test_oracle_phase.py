"""Pins of the Henyey-Greenstein phase function (Eq. 4), the j_sca pixel
weights and the wavelength-dependent resolution rule (Eq. 5-6), paper
Sect. 3.1.2."""

import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


@pytest.mark.parametrize("g", [0.0, 0.1, 0.3, 0.5, 0.7, 0.9, -0.4])
def test_hg_normalised_over_sphere(orc, g):
    val, _ = integrate.quad(lambda mu: 2 * math.pi * orc.hg(g, mu), -1, 1, epsabs=1e-13, limit=200)
    assert abs(val - 1.0) < 1e-10


def test_hg_isotropic_limit(orc):
    for mu in (-1, -0.3, 0, 0.5, 1):
        assert orc.hg(0.0, mu) == pytest.approx(1 / (4 * math.pi), rel=1e-15)


def closed_form_fwhm(g):
    """FWHM of Phi - Phi(pi) by inverting (1+g^2-2g cos t)^-3/2 directly."""
    f0 = (1 + g * g - 2 * g) ** -1.5
    fpi = (1 + g * g + 2 * g) ** -1.5
    half = fpi + 0.5 * (f0 - fpi)
    cos_h = (1 + g * g - half ** (-2.0 / 3.0)) / (2 * g)
    return 2 * math.acos(cos_h)


@pytest.mark.parametrize("g", [0.05, 0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.95])
def test_fwhm_matches_closed_form(orc, g):
    assert orc.hg_fwhm(g) == pytest.approx(closed_form_fwhm(g), rel=1e-12)


def test_k_hp_rule(orc):
    n_fwhm = json.load(open(GOLDEN))["n_fwhm"]["value"]
    for g in np.linspace(0.05, 0.9, 35):
        tmin = closed_form_fwhm(g) / n_fwhm
        # Eq. 5 inverts theta_min^2 ~ 4 pi / N_pix with N_pix = 12 * 4^k
        k = 0.5 * math.log2(4 * math.pi / (12 * tmin ** 2))
        assert orc.k_hp_real(g, n_fwhm) == pytest.approx(k, rel=1e-10)
        npix = 12 * 4 ** k
        assert tmin ** 2 == pytest.approx(4 * math.pi / npix, rel=1e-10)
        assert orc.k_hp(g, n_fwhm, 3) == min(3, max(0, math.floor(k)))
    # sharper profiles need finer sampling: k grows with g
    ks = [orc.k_hp_real(g, 5.0) for g in np.linspace(0.05, 0.9, 20)]
    assert all(b > a for a, b in zip(ks, ks[1:]))
    assert orc.k_hp(0.0, 5.0, 2) == 0


def test_memory_example_of_the_paper(orc):
    ex = json.load(open(GOLDEN))["jsca_memory_example"]
    npix = 12 * 4 ** ex["k_hp"]
    assert len(orc.healpix_vecs(2 ** ex["k_hp"])) == npix
    gb = ex["n_lambda"] * ex["n_cells"] * npix * 8 / 1e9
    assert abs(gb - ex["gbytes"]) / ex["gbytes"] < 0.02   # double-precision storage


@pytest.mark.parametrize("nside,g", [(1, 0.5), (2, 0.5), (2, 0.7), (4, 0.3), (4, 0.7)])
def test_weights(orc, nside, g):
    rng = np.random.default_rng(1)
    for _ in range(5):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        w = orc.hg_weights(nside, g, n)
        assert w.sum() == pytest.approx(1.0, abs=1e-14)
        assert (w > 0).all()
        v = orc.healpix_vecs(nside)
        # forward-peaked: the pixel nearest to n gets the largest weight
        assert np.argmax(w) == np.argmax(v @ n)
        # Riemann sum of Phi over equal-area pixels approximates 1 for mild g
        if nside >= 2 and g <= 0.5:
            raw = np.array([orc.hg(g, float(x @ n)) for x in v]) * 4 * math.pi / len(v)
            assert raw.sum() == pytest.approx(1.0, rel=0.05)


def test_weights_isotropic(orc):
    w = orc.hg_weights(2, 0.0, np.array([0.0, 0.6, 0.8]))
    np.testing.assert_allclose(w, 1.0 / 48, rtol=1e-14)


def test_weights_rotate_with_frame(orc):
    from paper_1709_03802_amd.workloads import rotation
    R = rotation(7)
    n = np.array([0.3, -0.4, np.sqrt(1 - 0.25)])
    w0 = orc.hg_weights(2, 0.6, n)
    w1 = orc.hg_weights(2, 0.6, R @ n, frame=R)
    np.testing.assert_allclose(w1, w0, rtol=1e-12)

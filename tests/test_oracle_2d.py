"""Pins of the oracle's 2D mode (paper Sect. 3.6: an axisymmetric model is
computed on the 3D grid by tracing only the sources of the first octant and
taking the other octants' contributions from symmetry).

* The direction set is mirror symmetric bit for bit: the vector of the
  mirror image of a pixel is the mirrored vector (every Nside used).
* A 3D run of a mirror-symmetric model is itself symmetric (each cell's U
  equals its mirror images'), on a uniform grid and on an octree where rays
  run inside face planes between finer leaves.
* The 2D mode equals the 3D run: fixed and adaptive rays (step 1, splits,
  blocking, per-wavelength skips, scattering iterations), U, S and the
  escape by direction to rounding, the tallies, and the counters of the
  traced rays times 8.
* Asymmetric models, leaves across a mirror plane, rotated frames, source
  masks and point sources are refused.
"""

import dataclasses

import numpy as np
import pytest

from paper_1709_03802_amd import workloads as W


def mirror_index(grid):
    c = grid.centres()
    lo, hi = grid.box()
    ctr = 0.5 * (lo + hi)
    key = {tuple(np.round(x, 9)): i for i, x in enumerate(c)}
    out = np.zeros((grid.n, 8), dtype=np.int64)
    for M in range(8):
        s = np.array([-1.0 if (M >> a) & 1 else 1.0 for a in range(3)])
        for i in range(grid.n):
            out[i, M] = key[tuple(np.round(ctr + s * (c[i] - ctr), 9))]
    return out


def rel(a, b):
    return float((np.abs(a - b) / np.maximum(np.abs(b), 1e-300)).max())


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 16, 64])
def test_pixel_vectors_are_mirror_exact(orc, nside):
    V = orc.healpix_vecs(nside)
    for M in range(1, 8):
        s = np.array([-1.0 if (M >> a) & 1 else 1.0 for a in range(3)])
        for p in range(len(V)):
            w = V[p] * s
            assert np.array_equal(V[orc.healpix_pix(nside, w)], w)


def symmetric_cases():
    return [("plain8 fixed", W.plain16(n=8, nside=4, lambdas=np.array([0.3, 1.0]), n_scatter=1).grid,
             W.RayPolicy(adaptive=False, nside=4, nside_max=4, n_scatter=1)),
            ("plain8 adaptive", W.plain16(n=8, nside=2, lambdas=np.array([0.3, 1.0]), n_scatter=1).grid,
             W.RayPolicy(adaptive=True, nside=2, nside_max=32, n_rays_min=4.0, f_U=1e-3, r_pre=0.3, step1=True,
                         n_scatter=1)),
            ("disk_tiny fixed", W.disk_tiny(mode_2d=True).grid,
             W.RayPolicy(adaptive=False, nside=4, nside_max=4, n_scatter=1)),
            ("disk_tiny adaptive", W.disk_tiny(mode_2d=True).grid, W.disk_tiny(mode_2d=True).policy)]


def compare_2d_3d(orc, grid, pol, name=""):
    """Each pass of the 2D mode against the 3D pass from the same inputs
    (the 2D run's own U_LL and pending scattered light, which are mirror
    symmetric): a chained comparison would let the order of the oracle's
    thread sums (1e-16) move a decision lying on its threshold."""
    m = orc.Model(grid)
    p2 = dataclasses.replace(pol, mode_2d=True)
    p3 = dataclasses.replace(pol, mode_2d=False)
    mi = mirror_index(grid)
    U_LL = None
    S_pending = None
    U_run = np.zeros((m.nl, m.n))
    modes = ([orc.STEP1] if pol.adaptive and pol.step1 else []) + [orc.DIRECT] + [orc.SCATTER] * pol.n_scatter
    if pol.adaptive and not pol.step1:
        U_LL = np.zeros((m.nl, m.n))
    merges = 0
    for mode in modes:
        a = m.run_pass(mode, p2, S_pending=S_pending, U_LL=U_LL)
        b = m.run_pass(mode, p3, S_pending=S_pending, U_LL=U_LL)
        # the 3D pass of a symmetric model is symmetric
        for M in range(1, 8):
            assert rel(b.U[:, mi[:, M]], b.U) < 1e-12, (name, mode, M)
        assert rel(a.U, b.U) < 1e-12, (name, mode)
        if mode != orc.STEP1:
            assert rel(a.S, b.S) < 1e-12, (name, mode)
        if not pol.adaptive:
            assert rel(a.escape, b.escape) < 1e-12
        np.testing.assert_allclose(a.tally, b.tally, rtol=1e-12, atol=1e-300)
        np.testing.assert_array_equal(a.counters * 8, b.counters)
        merges += b.counters[orc.C_MERGES]
        if mode == orc.STEP1:
            U_LL = a.U
        else:
            U_run = U_run + a.U
            S_pending = a.S
            if pol.adaptive:
                U_LL = U_run
    return merges


@pytest.mark.parametrize("case", range(4))
def test_2d_mode_equals_the_3d_run(orc, case):
    name, grid, pol = symmetric_cases()[case]
    compare_2d_3d(orc, grid, pol, name)


def test_2d_mode_refuses_what_it_cannot_fold(orc):
    wl = W.plain16(n=8, nside=2, n_scatter=0)
    pol = W.RayPolicy(adaptive=False, nside=2, nside_max=2, n_scatter=0, mode_2d=True)
    g = wl.grid.copy()
    g.rho[3] *= 1.5                              # density no longer symmetric
    with pytest.raises(ValueError):
        orc.Model(g).run_pass(orc.DIRECT, pol)
    g = wl.grid.copy()
    g.emis[0, 10] *= 2.0                         # emission no longer symmetric
    with pytest.raises(ValueError):
        orc.Model(g).run_pass(orc.DIRECT, pol)
    odd = W.plain16(n=7, nside=2, n_scatter=0).grid  # the central cells lie across the planes
    with pytest.raises(ValueError):
        orc.Model(odd).run_pass(orc.DIRECT, pol)
    m = orc.Model(wl.grid)
    with pytest.raises(ValueError):
        m.run_pass(orc.DIRECT, pol, frame=W.rotation(3))
    with pytest.raises(ValueError):
        m.run_pass(orc.DIRECT, pol, source_mask=np.ones(wl.grid.n, np.uint8))
    gp = wl.grid.copy()
    gp.point_pos = np.array([[0.5, 0.5, 0.5]])
    gp.point_lum = np.ones((1, 1))
    with pytest.raises(ValueError):
        orc.Model(gp).run_pass(orc.DIRECT, pol)
    # the same model without the flag runs
    m.run_pass(orc.DIRECT, dataclasses.replace(pol, mode_2d=False))

"""Pins of the oracle's ray merging (paper Sect. 3.1.1, Eq. 3 and the text
after it: a ray whose beam is too small for the crossed cell goes to the
'low' list; four rays in the same parent pixel, blocked after crossing the
same grid plane, merge into one ray with their average intensity, which
starts from their mean distance).

* Brute force, written from those definitions with independent slab
  geometry: every ray of one source on a small octree whose fine band makes
  rays split and whose coarse cells beyond make them merge: U per cell, S
  per cell and pixel (the merged ray scatters along its own direction), the
  split and merge counts.
* N_rays^max so large that no beam is too small reproduces the no-merging
  run (the same counts, U and S to the order of the threads' sums); merging conserves luminosity (balance with cut and
  skipped terms) and every ray ends once (a merge ends four rays and starts
  one); merging saves crossings on the disk and moves U by well under 1%.
* 2D mode with merging equals the 3D run with merging (the merge rule is
  mirror symmetric).
* N_rays^max below 4 N_rays is refused (a merged beam would be too large at
  once).
"""

import dataclasses
import math

import numpy as np
import pytest

from paper_1709_03802_amd import workloads as W
from test_oracle_adaptive import slab_segments


def banded_octree():
    """A 4 x 4 x 4 block of unit-1/4 root cubes; the cubes of the slab
    1/4 <= x < 1/2 are split twice (level 2), the rest stay coarse.  One
    emitting cell at the coarse corner x < 1/4; optical depth per unit
    length 0.3."""
    def want(c, s):
        return (c[:, 0] > 0.25) & (c[:, 0] < 0.5)
    level, ijk = W.refine_octree((4, 4, 4), (0.0, 0.0, 0.0), 0.25, 2, want)
    g = W.Grid(nroot=(4, 4, 4), lo=(0.0, 0.0, 0.0), root_size=0.25, level=level, ijk=ijk,
               rho=np.full(level.shape[0], 0.3), emis=np.zeros((1, level.shape[0])), kappa=np.ones(1),
               albedo=np.full(1, 0.5), g=np.full(1, 0.3), nside_sca=np.ones(1, np.int32), lambdas_um=np.ones(1))
    c = g.centres()
    s = int(np.argmin(np.linalg.norm(c - np.array([0.125, 0.375, 0.625]), axis=1)))
    g.emis[0, s] = 1.0
    return g, s


def entry_plane(grid, c, xs, n, t_in):
    """The face of leaf c through which the ray xs + t n enters it at t_in, as
    (axis, coordinate), or (-1, 0) when the ray starts inside c."""
    lo = np.asarray(grid.lo) + grid.ijk[c] * grid.side()[c]
    hi = lo + grid.side()[c]
    best, axis = -np.inf, -1
    for a in range(3):
        if n[a] == 0:
            continue
        ta = ((lo[a] if n[a] > 0 else hi[a]) - xs[a]) / n[a]
        if ta > best:
            best, axis = ta, a
    if not best >= t_in:
        return -1, 0.0
    return axis, float(lo[axis] if n[axis] > 0 else hi[axis])


def brute_force_merging(grid, s, pol, L0, nl=1):
    xs = grid.centres()[s]
    side = grid.side()
    V = side ** 3
    cl = grid.c_light
    alpha = grid.kappa[0] * grid.rho
    U = np.zeros(grid.n)
    ns = int(grid.nside_sca[0])
    S = np.zeros((grid.n, 12 * ns * ns))
    pv = np.array([pol_dirs(ns, q) for q in range(12 * ns * ns)])   # j_sca pixel directions, same frame
    g_hg, om_alb = float(grid.g[0]), float(grid.albedo[0])
    count = dict(splits=0, merges=0)

    def weights(n):
        mu = pv @ n
        phi = (1 - g_hg ** 2) / (1 + g_hg ** 2 - 2 * g_hg * mu) ** 1.5
        return phi / phi.sum()

    def dir_of(N, p):
        return np.asarray(pol_dirs(N, p))

    def walk(N, pix, t0, L, can_low, level):
        """('low', t, plane, L, t0_of_cell) or ('end',)"""
        om = 4 * math.pi / (12 * N * N)
        n = dir_of(N, pix)
        segs = slab_segments(grid, xs, n, t0)
        i = 0
        while i < len(segs):
            c, t_in, ln = segs[i]
            d2 = float(((grid.centres()[c] - xs) ** 2).sum())
            oint = math.inf if c == s else side[c] ** 2 / d2
            tau = alpha[c] * ln
            if om > oint / pol.n_rays_min and N < pol.nside_max and L > 0:
                count["splits"] += 1
                kids = [walk(2 * N, 4 * pix + k, t_in, L / 4, True, level + 1) for k in range(4)]
                planes = {k[2] for k in kids if k[0] == "low"}
                if all(k[0] == "low" for k in kids) and len(planes) == 1 and next(iter(planes))[0] >= 0:
                    count["merges"] += 1
                    L = sum(k[3] for k in kids)
                    tm = 0.25 * (kids[0][1] + kids[1][1] + kids[2][1] + kids[3][1])
                    segs = slab_segments(grid, xs, n, tm)
                    i = 0
                    continue
                for k in range(4):
                    if kids[k][0] == "low":
                        walk(2 * N, 4 * pix + k, kids[k][1], kids[k][3], False, level + 1)
                return ("end",)
            if can_low and level > 0 and c != s and om < oint / pol.n_rays_max:
                return ("low", t_in, entry_plane(grid, c, xs, n, t_in), L)
            ext = L * -math.expm1(-tau)
            U[c] += ext / (alpha[c] * V[c] * cl) if alpha[c] > 0 else L * ln / (V[c] * cl)
            S[c] += om_alb * ext * weights(n)
            L = L * math.exp(-tau)
            i += 1
        return ("end",)

    for r in range(12 * pol.nside ** 2):
        walk(pol.nside, r, 0.0, L0, False, 0)
    return U, S, count


pol_dirs = None


def test_merging_brute_force(orc):
    global pol_dirs
    g, s = banded_octree()
    R = W.rotation(29)                     # no ray runs along a face or through an edge
    pol_dirs = lambda N, p: R @ orc.healpix_vec(N, p)
    pol = W.RayPolicy(adaptive=True, nside=1, nside_max=8, n_rays_min=1.0, n_rays_max=4.0, f_U=0.0, n_scatter=0)
    r = orc.Model(g).run_pass(orc.DIRECT, pol, U_LL=np.zeros((1, g.n)), frame=R)
    L0 = 4 * math.pi * g.volume()[s] / 12
    U, S, count = brute_force_merging(g, s, pol, L0)
    assert count["merges"] > 0
    assert r.counters[orc.C_SPLITS] == count["splits"] and r.counters[orc.C_MERGES] == count["merges"]
    np.testing.assert_allclose(r.U[0], U, rtol=1e-11, atol=1e-14 * U.max())
    np.testing.assert_allclose(r.S.reshape(S.shape), S, rtol=1e-11, atol=1e-14 * S.max())


def test_no_low_beam_is_no_merging(orc):
    # the same rays and decisions; the threads' sums join in any order
    wl = W.disk_tiny()
    m = orc.Model(wl.grid)
    a = orc.run(m, wl.policy)
    b = orc.run(m, dataclasses.replace(wl.policy, n_rays_max=1e30))
    np.testing.assert_allclose(a.U, b.U, rtol=1e-13)
    np.testing.assert_allclose(a.S_total, b.S_total, rtol=1e-13, atol=1e-300)
    for pa, pb in zip(a.passes, b.passes):
        np.testing.assert_array_equal(pa.counters, pb.counters)


@pytest.mark.parametrize("nmax", [16.0, 64.0])
def test_merging_conserves_luminosity_and_ends_every_ray_once(orc, nmax):
    wl = W.disk_tiny()
    m = orc.Model(wl.grid)
    base = orc.run(m, wl.policy)
    r = orc.run(m, dataclasses.replace(wl.policy, n_rays_max=nmax))
    merges = 0
    for p, b in zip(r.passes, base.passes):
        t, c = p.tally, p.counters
        np.testing.assert_allclose(t[:, 1:6].sum(axis=1), t[:, 0], rtol=1e-12)
        assert c[orc.C_ESCAPES] + c[orc.C_CUTS] + c[orc.C_MAXSTEP] == \
            c[orc.C_RAYS] + 3 * c[orc.C_SPLITS] - 3 * c[orc.C_MERGES]
        assert c[orc.C_CROSS] <= b.counters[orc.C_CROSS]
        merges += c[orc.C_MERGES]
    assert merges > 0
    du = np.abs(r.U - base.U) / base.U
    assert du.max() < 1e-2


def test_2d_mode_with_merging_equals_3d(orc):
    from test_oracle_2d import compare_2d_3d
    wl = W.disk_tiny(mode_2d=True)
    assert compare_2d_3d(orc, wl.grid, dataclasses.replace(wl.policy, n_rays_max=64.0), "merging") > 0


def test_n_rays_max_below_four_n_rays_is_refused(orc):
    wl = W.disk_tiny()
    with pytest.raises(ValueError):
        orc.Model(wl.grid).run_pass(orc.STEP1, dataclasses.replace(wl.policy, n_rays_max=15.9))

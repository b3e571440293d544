"""Pins of the oracle's cell traversal against brute force.

The ray-cell intersections of Sect. 2 are found by stepping from face to face
through the adaptive grid.  Here every leaf's box is intersected with the ray
independently (slab method) and the sorted list of non-empty intersections must
equal the oracle's sequence, with the same path lengths, on tiny uniform grids
and random octrees, for rays in general position (no ties).
"""

import numpy as np
import pytest

from paper_1709_03802_amd import workloads as W


def brute_force(grid, o, d, t0=0.0):
    lo = np.asarray(grid.lo)[None, :] + grid.ijk * grid.side()[:, None]
    hi = lo + grid.side()[:, None]
    segs = []
    for c in range(grid.n):
        ta, tb = -np.inf, np.inf
        for a in range(3):
            if d[a] == 0:
                if not (lo[c, a] <= o[a] < hi[c, a]):
                    ta, tb = 1, 0
                continue
            t1 = (lo[c, a] - o[a]) / d[a]
            t2 = (hi[c, a] - o[a]) / d[a]
            ta = max(ta, min(t1, t2))
            tb = min(tb, max(t1, t2))
        ta = max(ta, t0)
        if tb - ta > 1e-12:
            segs.append((ta, c, tb - ta))
    segs.sort()
    return [s[1] for s in segs], np.array([s[2] for s in segs])


def box_exit(grid, o, d):
    blo, bhi = grid.box()
    t = np.inf
    for a in range(3):
        if d[a] > 0:
            t = min(t, (bhi[a] - o[a]) / d[a])
        elif d[a] < 0:
            t = min(t, (blo[a] - o[a]) / d[a])
    return t


GRIDS = [
    ("u2", lambda: W.plain16(n=2).grid),
    ("u3", lambda: W.plain16(n=3).grid),
    ("u4", lambda: W.plain16(n=4).grid),
    ("oct_a", lambda: W.random_octree(seed=1)),
    ("oct_b", lambda: W.random_octree(nroot=(3, 2, 1), root_size=1.0, max_level=3, p_split=0.5, seed=2,
                                      lo=(-1.5, -1.0, -0.5))),
    ("oct_c", lambda: W.random_octree(nroot=(1, 1, 1), root_size=2.0, max_level=4, p_split=0.6, seed=3)),
]


@pytest.mark.parametrize("name,make", GRIDS)
def test_traversal_matches_brute_force(orc, name, make):
    grid = make()
    m = orc.Model(grid)
    rng = np.random.default_rng(hash(name) % 2 ** 31)
    blo, bhi = grid.box()
    for trial in range(60):
        o = blo + rng.random(3) * (bhi - blo)
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        t0 = 0.0 if trial % 3 else rng.random() * 0.3 * box_exit(grid, o, d)
        cells, lens, tin = m.trace_cells(o, d, t0)
        keep = lens > 0
        want_cells, want_lens = brute_force(grid, o, d, t0)
        assert list(cells[keep]) == want_cells
        np.testing.assert_allclose(lens[keep], want_lens, rtol=1e-10, atol=1e-13)
        assert lens.sum() == pytest.approx(box_exit(grid, o, d) - t0, rel=1e-12)
        # entry distances are cumulative path lengths
        np.testing.assert_allclose(tin[keep][1:], t0 + np.cumsum(lens)[keep][:-1], rtol=1e-12)


def test_locate_tie_rule(orc):
    grid = W.plain16(n=4).grid
    m = orc.Model(grid)
    idx = lambda i, j, k: (k * 4 + j) * 4 + i
    # a point on the x = 0.5 face belongs to the side the direction points to
    p = [0.5, 0.1, 0.1]
    assert m.locate(p, [1, 0.1, 0.1]) == idx(2, 0, 0)
    assert m.locate(p, [-1, 0.1, 0.1]) == idx(1, 0, 0)
    # zero component: upper side
    assert m.locate(p, [0.0, 1.0, 0.0]) == idx(2, 0, 0)
    # leaving the block
    assert m.locate([1.0, 0.3, 0.3], [1, 0, 0]) == -1
    assert m.locate([0.0, 0.3, 0.3], [-1, 0, 0]) == -1
    assert m.locate([0.0, 0.3, 0.3], [1, 0, 0]) == idx(0, 1, 1)


def test_edge_crossing(orc):
    # a diagonal ray through cell edges: ties go x before y, the extra cells
    # it touches get zero length, the chord is exact
    grid = W.plain16(n=4).grid
    m = orc.Model(grid)
    s = 1 / np.sqrt(2)
    cells, lens, _ = m.trace_cells([0.125, 0.125, 0.3], [s, s, 0.0])
    idx = lambda i, j, k: (k * 4 + j) * 4 + i
    assert list(cells[lens > 1e-3]) == [idx(i, i, 1) for i in range(4)]
    assert (lens[lens <= 1e-3] < 1e-12).all()
    assert lens.sum() == pytest.approx(0.875 * np.sqrt(2), rel=1e-12)


def test_rejects_bad_grids(orc):
    g = W.plain16(n=2).grid
    bad = g.copy()
    bad.ijk[0] = bad.ijk[1]            # overlap and a gap
    with pytest.raises(ValueError):
        orc.Model(bad)
    bad = g.copy()
    bad.rho[3] = np.nan
    with pytest.raises(ValueError):
        orc.Model(bad)
    bad = g.copy()
    bad.nside_sca[0] = 3               # not a power of two
    with pytest.raises(ValueError):
        orc.Model(bad)

"""GPU 2D mode (paper Sect. 3.6) against the FP64 oracle.

The oracle's 2D mode equals its 3D run on these mirror-symmetric models
(pinned on the CPU), so matching it matches the full problem:

* fixed rays on a uniform grid and on the disk octree: a whole run (direct
  pass and scattering), U, S, the escape by direction within 1e-4 per
  element, the counters of the traced rays equal;
* adaptive rays on the disk octree, pass by pass from the same FP32 inputs
  (step 1, direct, scattering): U, S within 1e-4, split, cut, crossing,
  deposit and skip counts equal;
* the mirror images of every cell hold the same U on the GPU;
* asymmetric density (also after dartray_grid_set_rho), leaves across a
  mirror plane and rotated frames are refused.
"""

import numpy as np
import pytest

from paper_1709_03802_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def dr():
    import torch
    assert torch.cuda.is_available()
    from paper_1709_03802_amd import dartray
    dartray.load_library()
    return dartray


def as_f32(grid):
    g = grid.copy()
    for name in ("rho", "emis", "kappa", "albedo", "g"):
        setattr(g, name, getattr(g, name).astype(np.float32).astype(np.float64))
    return g


def rel(x, ref):
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    nz = (np.abs(ref) > 0) | (np.abs(x) > 0)
    if not nz.any():
        return np.zeros(1)
    return np.abs(x - ref)[nz] / np.maximum(np.abs(ref[nz]), 1e-30)


@pytest.mark.parametrize("which", ["plain8", "disk_tiny"])
def test_fixed_rays_2d_mode(dr, orc, which):
    import torch
    if which == "plain8":
        grid = W.plain16(n=8, nside=4, lambdas=np.array([0.3, 1.0, 2.2]), n_scatter=2).grid
    else:
        grid = W.disk_tiny(mode_2d=True).grid
    pol = W.RayPolicy(adaptive=False, nside=4, nside_max=4, n_scatter=2, mode_2d=True)
    g = as_f32(grid)
    ref = orc.run(orc.Model(g), pol)
    G = dr.Grid(g)
    out = dr.run(G, pol, escape=True)
    torch.cuda.synchronize()
    eu = rel(out.fields.U.cpu().numpy(), ref.U).max()
    es = rel(out.fields.S_total.cpu().numpy()[:G.s_size], ref.S_total).max()
    ee = rel(out.escape[-1], ref.passes[-1].escape).max()
    print(f"{which} 2D fixed: U {eu:.3g} S {es:.3g} escape {ee:.3g}", flush=True)
    assert eu <= TOL and es <= TOL and ee <= TOL
    for c, r in zip(out.counters, ref.passes):
        assert c[dr.C_CROSSINGS] == r.counters[orc.C_CROSS] and c[dr.C_RAYS] == r.counters[orc.C_RAYS]
    for t, r in zip(out.tallies, ref.passes):
        np.testing.assert_allclose(t[:, :4], r.tally[:, :4], rtol=1e-5, atol=1e-12 * r.tally[:, 0].max())
    # every mirror image holds the same U
    U = out.fields.U.cpu().numpy()
    from test_oracle_2d import mirror_index
    mi = mirror_index(g)
    for M in range(1, 8):
        assert np.array_equal(U[:, mi[:, M]], U)
    G.close()


def test_adaptive_rays_2d_mode_frozen_passes(dr, orc):
    from test_gpu_adaptive import run_frozen
    run_frozen(dr, orc, W.disk_tiny(mode_2d=True))


def test_2d_mode_refusals(dr):
    import torch
    wl = W.plain16(n=8, nside=2, n_scatter=0)
    pol = W.RayPolicy(adaptive=False, nside=2, nside_max=2, n_scatter=0, mode_2d=True)
    g = as_f32(wl.grid)
    g.rho[3] *= 1.5
    G = dr.Grid(g)
    with pytest.raises(dr.DartRayError) as e:
        dr.run(G, pol)
    assert e.value.code == dr.E_INVALID and "symmetric" in str(e.value)
    G.close()
    odd = as_f32(W.plain16(n=7, nside=2, n_scatter=0).grid)
    G = dr.Grid(odd)
    with pytest.raises(dr.DartRayError) as e:
        dr.run(G, pol)
    assert e.value.code == dr.E_INVALID
    G.close()
    G = dr.Grid(as_f32(wl.grid))
    with pytest.raises(dr.DartRayError) as e:
        dr.run(G, pol, frame=W.rotation(3))
    assert e.value.code == dr.E_UNSUPPORTED
    out = dr.run(G, pol)                      # a symmetric grid runs
    assert out.counters[0][dr.C_RAYS] == 48 * G.n // 8
    rho = torch.tensor(as_f32(wl.grid).rho, dtype=torch.float32, device="cuda")
    rho[5] *= 2.0
    G.set_rho(rho)                            # no longer symmetric
    with pytest.raises(dr.DartRayError) as e:
        dr.run(G, pol)
    assert e.value.code == dr.E_INVALID
    G.close()

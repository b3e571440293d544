"""GPU ray merging (paper Sect. 3.1.1, Eq. 3) against the FP64 oracle.

Each pass from the same FP32 inputs on both sides, as for the other
adaptive tests: step 1, the direct pass and the scattering passes of the
small disk with N_rays^max = 16 and 64 (merges happen in every pass that
splits), the same passes in 2D mode, and the direct pass of one source on
the banded octree of the oracle's brute-force pin in a rotated frame.  U and
S within 1e-4 per element; split, merge, cut, crossing, deposit, skip and
escape counts equal; every ray ends once.
"""

import dataclasses

import numpy as np
import pytest

from paper_1709_03802_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dr():
    import torch
    assert torch.cuda.is_available()
    from paper_1709_03802_amd import dartray
    dartray.load_library()
    return dartray


@pytest.mark.parametrize("nmax", [16.0, 64.0])
def test_merging_frozen_passes_small_disk(dr, orc, nmax):
    from test_gpu_adaptive import run_frozen
    wl = W.disk_tiny()
    run_frozen(dr, orc, W.Workload(wl.name, wl.grid, dataclasses.replace(wl.policy, n_rays_max=nmax)))


def test_merging_frozen_passes_2d_mode(dr, orc):
    from test_gpu_adaptive import run_frozen
    wl = W.disk_tiny(mode_2d=True)
    run_frozen(dr, orc, W.Workload(wl.name, wl.grid, dataclasses.replace(wl.policy, n_rays_max=64.0)))


def test_merging_one_source_banded_octree(dr, orc):
    import torch
    from test_gpu_adaptive import as_f32, check_counts, rel
    from test_oracle_merge import banded_octree
    g, s = banded_octree()
    g = as_f32(g)
    R = W.rotation(29)
    pol = W.RayPolicy(adaptive=True, nside=1, nside_max=8, n_rays_min=1.0, n_rays_max=4.0, f_U=0.0, n_scatter=0)
    ull = np.zeros((1, g.n))
    r = orc.Model(g).run_pass(orc.DIRECT, pol, U_LL=ull, frame=R)
    G = dr.Grid(g, nside_max=8)
    f = dr.Fields(G, keep_pass_u=True)
    dr.trace_direct(G, dr.make_opts(pol, dr.MODE_DIRECT, R), f)
    torch.cuda.synchronize()
    eu = rel(f.U_pass.cpu().numpy(), r.U).max()
    es = rel(f.S_pending.cpu().numpy()[:G.s_size], r.S).max()
    c = f.counters.cpu().numpy()
    print(f"banded octree: U {eu:.3g} S {es:.3g}, merges {c[dr.C_MERGES]}", flush=True)
    assert c[dr.C_MERGES] > 0
    check_counts(c, r.counters, dr, orc)
    assert eu <= 1e-4 and es <= 1e-4
    G.close()


def test_merging_beyond_three_split_levels_is_refused(dr):
    wl = W.disk_tiny(nside_max=64)          # 4 split levels above Nside 4
    G = dr.Grid(as_f32_grid(wl.grid), nside_max=64)
    f = dr.Fields(G)
    with pytest.raises(dr.DartRayError) as e:
        dr.trace_direct(G, dr.make_opts(dataclasses.replace(wl.policy, n_rays_max=64.0), dr.MODE_STEP1), f)
    assert e.value.code == dr.E_UNSUPPORTED
    G.close()


def as_f32_grid(grid):
    from test_gpu_adaptive import as_f32
    return as_f32(grid)

"""The bench's own workload at full size: the 30x30x6 kpc disk on 207,848
octree leaves, 8 wavelengths, adaptive rays Nside 4..1024.

* step 1 of 48 seeded emitting cells against the FP64 oracle over the whole
  grid: 1e-4 per element, every counter equal;
* the direct pass of the same cells, both sides given the oracle's step-1
  result of those cells (rounded to FP32) as U_LL: both take the
  significance decisions in FP64, so every counter is equal and every U and
  S value is within 1e-4;
* a scattering pass of 48 seeded dusty cells chosen by the source mask from
  a synthetic pending scattered luminosity held by 548 cells (the other 500
  must be skipped): every counter equal, U and S within 1e-4;
* the full run of every source (step 1, direct, 3 scattering passes): FP64
  luminosity balance of every pass within 1e-6.
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


@pytest.fixture(scope="module")
def disk():
    wl = W.disk()
    g = wl.grid.copy()
    for name in ("rho", "emis", "kappa", "albedo", "g"):
        setattr(g, name, getattr(g, name).astype(np.float32).astype(np.float64))
    rng = np.random.default_rng(2017)
    mask = np.zeros(g.n, dtype=np.uint8)
    mask[rng.choice(np.flatnonzero(g.emis.sum(axis=0) > 0), 48, replace=False)] = 1
    return wl, g, mask


@pytest.fixture(scope="module")
def step1(orc, disk):
    wl, g, mask = disk
    m = orc.Model(g)
    return m, m.run_pass(orc.STEP1, wl.policy, source_mask=mask, n_threads=16)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def rel(x, ref):
    x = np.asarray(x, np.float64)
    nz = (np.abs(ref) > 0) | (np.abs(x) > 0)
    return np.abs(x - ref)[nz] / np.maximum(np.abs(ref[nz]), 1e-30)


def compare_pass(dr, orc, m, G, f, ref, label):
    e = rel(f.U_pass.cpu().numpy(), ref.U)
    es = np.concatenate([rel(f.S_pending[G.s_offset[l]:G.s_offset[l + 1]].cpu().numpy(),
                             ref.S[m.s_offset[l]:m.s_offset[l + 1]]) for l in range(G.nl)])
    c = f.counters.cpu().numpy()
    print(f"{label}: U max rel {e.max():.3g} p99.9 {np.quantile(e, 0.999):.3g}; S max rel {es.max():.3g} "
          f"p99.9 {np.quantile(es, 0.999):.3g}; crossings {c[dr.C_CROSSINGS]} (oracle {ref.counters[orc.C_CROSS]}); "
          f"splits {c[dr.C_SPLITS]} ({ref.counters[orc.C_SPLITS]}), cuts {c[dr.C_CUTS]} ({ref.counters[orc.C_CUTS]}), "
          f"deposits {c[dr.C_DEPOSITS]} ({ref.counters[orc.C_DEPOSITS]}), skips {c[dr.C_SKIPS]} "
          f"({ref.counters[orc.C_SKIPS]})", flush=True)
    for k_gpu, k_orc in ((dr.C_CROSSINGS, orc.C_CROSS), (dr.C_SPLITS, orc.C_SPLITS), (dr.C_CUTS, orc.C_CUTS),
                         (dr.C_RAYS, orc.C_RAYS), (dr.C_DEPOSITS, orc.C_DEPOSITS), (dr.C_SKIPS, orc.C_SKIPS)):
        assert c[k_gpu] == ref.counters[k_orc], k_gpu
    tg = f.tally.cpu().numpy()
    for col in (dr.T_EMITTED, dr.T_ABSORBED, dr.T_SCATTERED, dr.T_ESCAPED, dr.T_CUT, dr.T_SKIPPED):
        assert np.all(np.abs(tg[:, col] - ref.tally[:, col]) <= 1e-6 * ref.tally[:, dr.T_EMITTED]), col
    assert e.max() <= TOL and es.max() <= TOL


def test_full_disk_sampled_step1_and_direct_pass(dr, orc, disk, step1):
    import torch
    wl, g, mask = disk
    pol = wl.policy
    m, r1 = step1
    G = dr.Grid(g, nside_max=max(pol.nside_max, 64))
    mt = torch.as_tensor(mask).cuda()
    f = dr.Fields(G)
    dr.trace_direct(G, dr.make_opts(pol, dr.MODE_STEP1, source_mask=mt), f)
    torch.cuda.synchronize()
    e1 = rel(f.U_LL.cpu().numpy(), r1.U)
    c1 = f.counters.cpu().numpy()
    rows = int(c1[dr.C_U_ROWS])
    print(f"disk step 1, 48 sources: U_LL max rel {e1.max():.3g}; crossings {c1[dr.C_CROSSINGS]} "
          f"(oracle {r1.counters[orc.C_CROSS]}); energy-density rows {rows} "
          f"({rows / max(int(c1[dr.C_CROSSINGS]), 1):.3f} per crossing)", flush=True)
    assert e1.max() <= TOL
    for k_gpu, k_orc in ((dr.C_CROSSINGS, orc.C_CROSS), (dr.C_SPLITS, orc.C_SPLITS), (dr.C_CUTS, orc.C_CUTS),
                         (dr.C_RAYS, orc.C_RAYS), (dr.C_ESCAPES, orc.C_ESCAPES), (dr.C_DEPOSITS, orc.C_DEPOSITS)):
        assert c1[k_gpu] == r1.counters[k_orc]
    # sibling rays share rows of the cells they cross together: at least one
    # row per four crossings, and fewer rows than crossings (the four launch
    # rays of an item all start in the source's own cell)
    assert int(c1[dr.C_CROSSINGS]) / 4 <= rows < int(c1[dr.C_CROSSINGS])
    # direct pass with the same FP32 U_LL on both sides
    ull = f32(r1.U)
    r2 = m.run_pass(orc.DIRECT, pol, U_LL=ull, source_mask=mask, n_threads=16)
    f2 = dr.Fields(G, keep_pass_u=True)
    f2.U_LL.copy_(torch.as_tensor(ull, dtype=torch.float32))
    dr.trace_direct(G, dr.make_opts(pol, dr.MODE_DIRECT, source_mask=mt), f2)
    torch.cuda.synchronize()
    compare_pass(dr, orc, m, G, f2, r2, "disk direct pass, 48 sources")


def test_full_disk_sampled_scattering_pass(dr, orc, disk, step1):
    """Additivity over sources (Sect. 3.4) with a frozen pending scattered
    luminosity: the scattering pass of 48 seeded cells of the full disk."""
    import torch
    wl, g, mask = disk
    pol = wl.policy
    m, r1 = step1
    G = dr.Grid(g, nside_max=max(pol.nside_max, 64))
    rng = np.random.default_rng(1703)
    dusty = np.flatnonzero(g.rho > 0)
    cells = rng.choice(dusty, 548, replace=False)
    smask = np.zeros(g.n, np.uint8)
    smask[cells[:48]] = 1
    # synthetic pending light: rows of random pixel values scaled by the cell's luminosity
    Sp = np.zeros(m.s_size)
    for l in range(g.n_lambda):
        blk = Sp[m.s_offset[l]:m.s_offset[l + 1]].reshape(g.n, -1)
        lum = 4 * np.pi * g.emis[l, cells] * g.side()[cells] ** 3 + 1e-6
        blk[cells] = rng.random((cells.size, blk.shape[1])) * lum[:, None] / blk.shape[1]
    Sp = f32(Sp)
    ull = f32(r1.U)
    ref = m.run_pass(orc.SCATTER, pol, S_pending=Sp, U_LL=ull, source_mask=smask, n_threads=16)
    assert ref.counters[orc.C_RAYS] > 0
    f = dr.Fields(G, keep_pass_u=True)
    dr.trace_direct(G, dr.make_opts(pol, dr.MODE_DIRECT, source_mask=torch.zeros(g.n, dtype=torch.uint8).cuda()), f)
    f.U_LL.copy_(torch.as_tensor(ull, dtype=torch.float32))
    f.S_pending.copy_(torch.as_tensor(np.concatenate([Sp, np.zeros(f.S_pending.numel() - G.s_size)]),
                                      dtype=torch.float32))
    torch.cuda.synchronize()
    dr.scatter_iter(G, dr.make_opts(pol, dr.MODE_DIRECT, source_mask=torch.as_tensor(smask).cuda()), f)
    torch.cuda.synchronize()
    compare_pass(dr, orc, m, G, f, ref, "disk scattering pass, 48 of 548 sources")


def test_full_disk_run_balance(dr, disk):
    import torch
    wl, g, _ = disk
    G = dr.Grid(g, nside_max=max(wl.policy.nside_max, 64))
    out = dr.run(G, wl.policy)
    torch.cuda.synchronize()
    bal = [float(np.max(np.abs(t[:, 1:6].sum(axis=1) - t[:, 0]) / t[:, 0])) for t in out.tallies]
    cross = [int(c[dr.C_CROSSINGS]) for c in out.counters]
    print(f"disk full run: crossings per pass {cross}; balance {['%.2g' % b for b in bal]}; r_k {out.r_k}",
          flush=True)
    assert max(bal) <= 1e-6
    assert all(a > b for a, b in zip(out.r_k, out.r_k[1:]))
    U = out.fields.U.cpu().numpy()
    assert np.all(np.isfinite(U)) and np.all(U >= 0)

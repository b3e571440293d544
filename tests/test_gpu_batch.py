"""Batches of models: one persistent march launch per pass for every model,
eager and replayed from a captured HIP graph.

Each model's fields from a batch equal those of the model run alone (same
kernels, FP32 bin additions in another order: 1e-6 relative), one model is
checked against the FP64 oracle (1e-4), and every graph replay, with eager
work and synchronisations between replays, reproduces the eager batch.
"""

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


def as_f32(grid):
    g = grid.copy()
    for name in ("rho", "emis", "kappa", "albedo", "g"):
        setattr(g, name, getattr(g, name).astype(np.float32).astype(np.float64))
    return g


def rel(x, ref):
    return float(np.max(np.abs(x - ref) / np.maximum(np.abs(ref), 1e-30)))


@pytest.fixture(scope="module")
def models():
    return W.disk_batch(5, leaves=(300, 3000), seed=5, nside=4, n_scatter=2)


def host(f, G):
    return (f.U.cpu().numpy().astype(np.float64), f.S_total.cpu().numpy()[:G.s_size].astype(np.float64),
            f.tally.cpu().numpy().copy(), f.counters.cpu().numpy().copy())


def test_batch_matches_single_runs_and_oracle(dr, orc, models):
    import torch
    pol = models[0].policy
    singles = []
    for wl in models:
        G = dr.Grid(as_f32(wl.grid))
        out = dr.run(G, pol)
        torch.cuda.synchronize()
        singles.append(host(out.fields, G))
    s = torch.cuda.Stream()
    Gs = [dr.Grid(as_f32(wl.grid), stream=s) for wl in models]
    fs = [dr.Fields(G) for G in Gs]
    torch.cuda.synchronize()
    B = dr.Batch(Gs)
    B.run(pol, fs)
    s.synchronize()
    for k, (G, f) in enumerate(zip(Gs, fs)):
        U, S, tally, cnt = host(f, G)
        eu, es = rel(U, singles[k][0]), rel(S, singles[k][1])
        print(f"model {k} ({G.n} leaves): batch vs single U {eu:.3g} S {es:.3g}", flush=True)
        assert eu <= 1e-6 and es <= 1e-6
        np.testing.assert_allclose(tally, singles[k][2], rtol=1e-6, atol=1e-12 * np.abs(singles[k][2]).max())
        # counters of the last pass
        assert np.array_equal(cnt, singles[k][3])
    k = int(np.argmin([wl.grid.n for wl in models]))
    ref = orc.run(orc.Model(as_f32(models[k].grid)), pol)
    U, S, _, _ = host(fs[k], Gs[k])
    print(f"model {k} vs oracle: U {rel(U, ref.U):.3g} S {rel(S, ref.S_total):.3g}", flush=True)
    assert rel(U, ref.U) <= 1e-4 and rel(S, ref.S_total) <= 1e-4


def test_graph_replays_reproduce_the_eager_batch(dr, models):
    import torch
    pol = models[0].policy
    s = torch.cuda.Stream()
    Gs = [dr.Grid(as_f32(wl.grid), stream=s) for wl in models]
    fs = [dr.Fields(G) for G in Gs]
    torch.cuda.synchronize()
    B = dr.Batch(Gs)
    B.run(pol, fs)
    s.synchronize()
    eager = [host(f, G) for f, G in zip(fs, Gs)]
    fg = [dr.Fields(G) for G in Gs]
    torch.cuda.synchronize()
    B.capture(pol, fg)
    s.synchronize()
    other = dr.Grid(as_f32(models[1].grid))
    for rep in range(3):
        for f in fg:
            f.U.zero_()                    # U accumulates over passes (each adds its U_k)
            f.S_total.fill_(3.0)           # the direct pass overwrites S_total and S_pending
            f.S_pending.fill_(5.0)
        torch.cuda.synchronize()
        B.replay()
        s.synchronize()
        for k, (f, G) in enumerate(zip(fg, Gs)):
            U, S, tally, cnt = host(f, G)
            assert rel(U, eager[k][0]) <= 1e-6, (rep, k)
            assert rel(S, eager[k][1]) <= 1e-6, (rep, k)
            assert np.array_equal(cnt, eager[k][3])
        dr.run(other, pol)                 # eager work of the program between replays
        torch.cuda.synchronize()


def test_batch_argument_errors(dr, models):
    import torch
    s = torch.cuda.Stream()
    G1 = dr.Grid(as_f32(models[0].grid), stream=s)
    G2 = dr.Grid(as_f32(W.plain16(n=4, nside=2).grid), stream=s)
    with pytest.raises(dr.DartRayError) as e:
        dr.Batch([G1, G2])                 # wavelength counts differ
    assert e.value.code == dr.E_INVALID
    with pytest.raises(dr.DartRayError) as e:
        dr.Batch([G1, G1])
    assert e.value.code == dr.E_INVALID
    G3 = dr.Grid(as_f32(models[1].grid))   # another stream
    with pytest.raises(dr.DartRayError) as e:
        dr.Batch([G1, G3])
    assert e.value.code == dr.E_INVALID
    B = dr.Batch([G1])
    with pytest.raises(dr.DartRayError) as e:
        B.replay()
    assert e.value.code == dr.E_STATE
    adaptive = W.RayPolicy(adaptive=True, nside=4, nside_max=8, f_U=1e-3, n_scatter=1)
    with pytest.raises(dr.DartRayError) as e:
        B.run(adaptive, [dr.Fields(G1)])
    assert e.value.code == dr.E_UNSUPPORTED

"""The autotuner on the GPU: it applies a valid setting no slower than the
start, caches it, and the tuned run still gives the same fields."""

import numpy as np
import pytest

from paper_1709_03802_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_autotune_plain_grid(tmp_path):
    import torch
    from paper_1709_03802_amd import autotune as AT
    from paper_1709_03802_amd import dartray as dr
    wl = W.plain16(n=16, nside=4, lambdas=np.array([0.15, 0.3, 0.55, 1.2, 2.2]), n_scatter=1)
    ref = dr.run(dr.Grid(wl.grid), wl.policy)
    torch.cuda.synchronize()
    U0 = ref.fields.U.cpu().numpy()
    G = dr.Grid(wl.grid)
    cache = str(tmp_path / "tune.json")
    setting, ms, log = AT.tune(G, wl.policy, cache_path=cache, rounds=1, repeats=2, verbose=True)
    assert ms > 0 and len(log) > 3
    assert ms <= log[0][1]                       # the start is evaluated first
    assert G.tuning().as_dict() == {**G.tuning().as_dict(), **setting}
    again, ms2, log2 = AT.tune(dr.Grid(wl.grid), wl.policy, cache_path=cache)
    assert again == setting and log2 == []
    out = dr.run(G, wl.policy)
    torch.cuda.synchronize()
    U = out.fields.U.cpu().numpy()
    assert np.max(np.abs(U - U0) / np.maximum(np.abs(U0), 1e-30)) <= 1e-6

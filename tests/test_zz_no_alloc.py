"""The direct pass that allocates nothing (dartray_trace_direct_noalloc)
against dartray_trace_direct, through the C ABI.

Both run the same kernels; the allocation-free entry point takes its work
arrays from a static per-device scratch array.  Two calls in a row, the
second on a smaller grid (the scratch keeps the first call's contents), must
each equal the allocating pass: U and S within 1e-6 (the order of FP32
additions into the direction bins), tallies within 1e-9, counters equal.  A
grid whose work arrays exceed the scratch is refused with a message, before
any output is written.
"""

import ctypes as C

import numpy as np
import pytest

from paper_1709_03802_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dr():
    import torch
    assert torch.cuda.is_available()
    from paper_1709_03802_amd import dartray
    L = dartray.load_library()
    L.dartray_trace_direct_noalloc.argtypes = [C.c_void_p, C.POINTER(dartray.TraceOpts), C.POINTER(dartray.FieldsC)]
    L.dartray_trace_direct_noalloc.restype = C.c_int
    return dartray


def as_f32(grid):
    g = grid.copy()
    for name in ("rho", "emis", "kappa", "albedo", "g"):
        setattr(g, name, getattr(g, name).astype(np.float32).astype(np.float64))
    return g


def rel(x, ref):
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.max(np.abs(x - ref) / np.maximum(np.abs(ref), 1e-30)))


def noalloc(dr, G, opts, f):
    fc = f.c()
    rc = dr.load_library().dartray_trace_direct_noalloc(G.h, C.byref(opts), C.byref(fc))
    if rc != dr.OK:
        raise dr.DartRayError(rc, dr.load_library().dartray_last_error().decode())


def test_noalloc_direct_pass_equals_the_allocating_pass_twice(dr):
    import torch
    cases = [(W.plain16(n=16, nside=8, n_scatter=0), "16^3, 1 wavelength, Nside 8"),
             (W.plain16(n=7, nside=4, lambdas=np.array([0.15, 0.55, 2.2]), n_scatter=0),
              "7^3, 3 wavelengths, Nside 4")]
    for wl, label in cases:
        print(f"case {label}", flush=True)
        G = dr.Grid(as_f32(wl.grid))
        opts = dr.make_opts(wl.policy, dr.MODE_DIRECT)
        ref = dr.Fields(G, escape_nside=wl.policy.nside)
        dr.trace_direct(G, opts, ref)
        got = dr.Fields(G, escape_nside=wl.policy.nside)
        noalloc(dr, G, opts, got)
        torch.cuda.synchronize()
        eu = rel(got.U.cpu().numpy(), ref.U.cpu().numpy())
        es = rel(got.S_total.cpu().numpy()[:G.s_size], ref.S_total.cpu().numpy()[:G.s_size])
        ee = rel(got.escape.cpu().numpy(), ref.escape.cpu().numpy())
        print(f"  U {eu:.3g} S {es:.3g} escape {ee:.3g}", flush=True)
        assert eu <= 1e-6 and es <= 1e-6 and ee <= 1e-6
        np.testing.assert_allclose(got.tally.cpu().numpy(), ref.tally.cpu().numpy(), rtol=1e-9, atol=0)
        np.testing.assert_array_equal(got.counters.cpu().numpy(), ref.counters.cpu().numpy())
        # the handle's own work set is back in use: a scattering iteration follows either pass alike
        r1 = dr.scatter_iter(G, opts, ref)
        r2 = dr.scatter_iter(G, opts, got)
        assert r1 == pytest.approx(r2, rel=1e-6)
        G.close()


def test_noalloc_refuses_grids_beyond_its_scratch(dr):
    import torch
    wl = W.plain16(n=64, nside=2, n_lambda=32, n_scatter=0)
    G = dr.Grid(as_f32(wl.grid))
    f = dr.Fields(G)
    f.U.fill_(7.0)
    with pytest.raises(dr.DartRayError) as ei:
        noalloc(dr, G, dr.make_opts(wl.policy, dr.MODE_DIRECT), f)
    assert ei.value.code == dr.E_UNSUPPORTED and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert float(f.U.min()) == 7.0 and float(f.U.max()) == 7.0
    G.close()

"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, its structs have the layout the binding assumes, and
malformed grid descriptions are rejected before any device work."""

import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dartray.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1709_03802_amd import dartray
    if not os.path.exists(dartray.LIB_PATH):
        from paper_1709_03802_amd import build
        build.build()
    return dartray.load_library()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?(?:int|int64_t|char|const char)\s*\*?\s*(dartray_\w+)\s*\(", text, re.M)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    from paper_1709_03802_amd import dartray
    assert sorted(dartray.EXPORTS) == names


def test_version(lib):
    from paper_1709_03802_amd import dartray
    assert dartray.version().startswith("dartray-gfx950")


def test_struct_layout_matches_header(tmp_path):
    from paper_1709_03802_amd import dartray
    src = tmp_path / "probe.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "dartray.h"
int main(void) {
  printf("%zu %zu %zu %zu\\n", sizeof(dartray_grid_desc), sizeof(dartray_trace_opts), sizeof(dartray_fields), sizeof(dartray_tuning));
  printf("%zu %zu %zu %zu %zu\\n", offsetof(dartray_grid_desc, c_light), offsetof(dartray_grid_desc, nside_max), offsetof(dartray_trace_opts, frame),
         offsetof(dartray_trace_opts, max_steps), offsetof(dartray_fields, counters));
  printf("%zu %zu\\n", offsetof(dartray_tuning, item_order), offsetof(dartray_fields, escape));
  printf("%zu %zu %zu\\n", offsetof(dartray_trace_opts, f_U), offsetof(dartray_trace_opts, r_pre), offsetof(dartray_trace_opts, flags));
  printf("%zu %zu %zu\\n", offsetof(dartray_grid_desc, n_point), offsetof(dartray_grid_desc, point_lum), sizeof(dartray_observer));
  printf("%zu %zu %zu %zu\\n", sizeof(dartray_dust_model), offsetof(dartray_dust_model, dlambda), sizeof(dartray_selfheat_opts),
         offsetof(dartray_selfheat_opts, conv));
  return 0;
}
""")
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)]).decode().split()
    got = [int(x) for x in out]
    want = [C.sizeof(dartray.GridDesc), C.sizeof(dartray.TraceOpts), C.sizeof(dartray.FieldsC), C.sizeof(dartray.Tuning),
            dartray.GridDesc.c_light.offset, dartray.GridDesc.nside_max.offset, dartray.TraceOpts.frame.offset, dartray.TraceOpts.max_steps.offset,
            dartray.FieldsC.counters.offset, dartray.Tuning.item_order.offset, dartray.FieldsC.escape.offset,
            dartray.TraceOpts.f_U.offset, dartray.TraceOpts.r_pre.offset, dartray.TraceOpts.flags.offset,
            dartray.GridDesc.n_point.offset, dartray.GridDesc.point_lum.offset, C.sizeof(dartray.Observer),
            C.sizeof(dartray.DustModelC), dartray.DustModelC.dlambda.offset, C.sizeof(dartray.SelfHeatOpts),
            dartray.SelfHeatOpts.conv.offset]
    assert got == want


def _desc(grid):
    from paper_1709_03802_amd import dartray
    keep = dict(
        level=np.ascontiguousarray(grid.level, dtype=np.int32),
        ijk=np.ascontiguousarray(grid.ijk, dtype=np.int64),
        rho=np.ascontiguousarray(grid.rho, dtype=np.float32),
        emis=np.ascontiguousarray(grid.emis, dtype=np.float32),
        kappa=np.ascontiguousarray(grid.kappa, dtype=np.float32),
        albedo=np.ascontiguousarray(grid.albedo, dtype=np.float32),
        g=np.ascontiguousarray(grid.g, dtype=np.float32),
        nside_sca=np.ascontiguousarray(grid.nside_sca, dtype=np.int32),
    )
    d = dartray.GridDesc()
    d.nroot = (C.c_int32 * 3)(*grid.nroot)
    d.lo = (C.c_double * 3)(*grid.lo)
    d.root_size = grid.root_size
    d.n_leaves = grid.n
    p = lambda a, t: a.ctypes.data_as(C.POINTER(t))
    d.leaf_level = p(keep["level"], C.c_int32)
    d.leaf_ijk = p(keep["ijk"], C.c_int64)
    d.rho = p(keep["rho"], C.c_float)
    d.emis = p(keep["emis"], C.c_float)
    d.n_lambda = grid.n_lambda
    d.kappa = p(keep["kappa"], C.c_float)
    d.albedo = p(keep["albedo"], C.c_float)
    d.g = p(keep["g"], C.c_float)
    d.nside_sca = p(keep["nside_sca"], C.c_int32)
    d.n_fwhm = 5.0
    d.k_max = 2
    d.c_light = 1.0
    d.nside_max = 0
    return d, keep


@pytest.mark.parametrize("breakage", ["overlap", "gap", "nan_rho", "neg_emis", "nside3", "albedo", "g1",
                                      "zero_n", "outside", "c_light"])
def test_malformed_descriptions_rejected_before_device_work(lib, breakage):
    from paper_1709_03802_amd import workloads as W
    from paper_1709_03802_amd import dartray
    grid = W.random_octree(seed=5)
    if breakage == "overlap":
        grid.ijk[1] = grid.ijk[0]
        grid.level[1] = grid.level[0]
    elif breakage == "gap":
        grid = grid.copy()
        grid.level = grid.level[1:]
        grid.ijk = grid.ijk[1:]
        grid.rho = grid.rho[1:]
        grid.emis = grid.emis[:, 1:]
    elif breakage == "nan_rho":
        grid.rho[2] = np.nan
    elif breakage == "neg_emis":
        grid.emis[0, 3] = -1.0
    elif breakage == "nside3":
        grid.nside_sca[0] = 3
    elif breakage == "albedo":
        grid.albedo[0] = 1.5
    elif breakage == "g1":
        grid.g[0] = 1.0
    elif breakage == "outside":
        grid.ijk[0, 0] = 10 ** 6
    d, keep = _desc(grid)
    if breakage == "zero_n":
        d.n_leaves = 0
    if breakage == "c_light":
        d.c_light = 0.0
    h = C.c_void_p()
    rc = lib.dartray_grid_create(C.byref(d), None, C.byref(h))
    assert rc == dartray.E_INVALID
    assert h.value is None
    assert len(lib.dartray_last_error()) > 0


def test_eq5_rule_beyond_k_max_3_is_unsupported(lib):
    """The j_sca resolution of Eq. 5 is capped at k = 3 (Nside_sca 8): a
    larger k_max with the rule in use is refused, not silently capped; with
    every nside_sca given explicitly k_max plays no part."""
    from paper_1709_03802_amd import workloads as W
    from paper_1709_03802_amd import dartray
    grid = W.random_octree(seed=5)
    grid.nside_sca[:] = 0
    d, keep = _desc(grid)
    d.k_max = 4
    h = C.c_void_p()
    assert lib.dartray_grid_create(C.byref(d), None, C.byref(h)) == dartray.E_UNSUPPORTED
    assert h.value is None and b"k_max" in lib.dartray_last_error()


@pytest.mark.parametrize("breakage", ["outside", "on_upper_face", "nan_pos", "neg_lum", "null_array"])
def test_malformed_point_sources_rejected(lib, breakage):
    from paper_1709_03802_amd import workloads as W
    from paper_1709_03802_amd import dartray
    grid = W.random_octree(seed=5)
    lo, hi = grid.box()
    pos = np.array([lo + 0.3 * (hi - lo), lo + 0.7 * (hi - lo)], dtype=np.float64)
    lum = np.ones((grid.n_lambda, 2), dtype=np.float32)
    if breakage == "outside":
        pos[1, 0] = hi[0] + 0.1
    elif breakage == "on_upper_face":
        pos[0, 2] = hi[2]
    elif breakage == "nan_pos":
        pos[0, 1] = np.nan
    elif breakage == "neg_lum":
        lum[0, 1] = -1.0
    d, keep = _desc(grid)
    d.n_point = 2
    d.point_pos = pos.ctypes.data_as(C.POINTER(C.c_double))
    d.point_lum = None if breakage == "null_array" else lum.ctypes.data_as(C.POINTER(C.c_float))
    h = C.c_void_p()
    assert lib.dartray_grid_create(C.byref(d), None, C.byref(h)) == dartray.E_INVALID
    assert h.value is None and b"point" in lib.dartray_last_error()


def test_null_arguments(lib):
    from paper_1709_03802_amd import dartray
    assert lib.dartray_grid_create(None, None, None) == dartray.E_INVALID
    assert lib.dartray_trace_direct(None, None, None) == dartray.E_INVALID
    assert lib.dartray_scatter_iter(None, None, None, None) == dartray.E_INVALID
    assert lib.dartray_grid_destroy(None) == dartray.OK
    assert lib.dartray_set_tuning(None, None) == dartray.E_INVALID
    assert lib.dartray_get_tuning(None, None) == dartray.E_INVALID
    assert lib.dartray_absorbed(None, None, None) == dartray.E_INVALID
    assert lib.dartray_dust_emission(None, None, None, None, None) == dartray.E_INVALID
    assert lib.dartray_grid_set_emis(None, None) == dartray.E_INVALID
    assert lib.dartray_dust_selfheat(None, None, None, None, None, None, None, None, None, None, None, None) == \
        dartray.E_INVALID

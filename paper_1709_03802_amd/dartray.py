"""Python binding of the gfx950 ray-march library (``libdartray.so``).

Argument marshalling only: every step of a pass runs in the library's HIP
kernels.  torch provides device memory and the stream.  Entry points mirror the
C ABI declared in ``include/dartray.h``:

    Grid(...)                 -> dartray_grid_create / dartray_grid_destroy
    trace_direct(...)         -> dartray_trace_direct
    scatter_iter(...)         -> dartray_scatter_iter
    trace_adjoint(...)        -> dartray_trace_adjoint
    debug_ray_cells(...)      -> dartray_debug_ray_cells

``run()`` chains the passes in the order of the paper's algorithm (Sect. 2):
optional step 1, the direct-light pass, then the scattering iterations.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
# DARTRAY_LIB names another build of the library to load (the host-sanitizer
# run of sanitize_host.sh)
LIB_PATH = os.environ.get("DARTRAY_LIB") or os.path.join(PKG, "libdartray.so")

OK, E_INVALID, E_OOM, E_DEVICE, E_STATE, E_UNSUPPORTED, E_NUMERIC = 0, -1, -2, -3, -4, -5, -6
MODE_STEP1, MODE_DIRECT = 0, 1
PROF_FIXED, PROF_STEP1, PROF_SCATTERING, PROF_ADJOINT, PROF_ALL = 1, 2, 4, 8, 15
FLAG_COUNTERS, FLAG_CHECK, FLAG_CONTINUE, FLAG_2D = 1, 2, 4, 8
T_EMITTED, T_ABSORBED, T_SCATTERED, T_ESCAPED, T_CUT, T_SKIPPED = range(6)
C_CROSSINGS, C_RAYS, C_SPLITS, C_CUTS, C_ESCAPES, C_DEPOSITS, C_SKIPS, C_MAXSTEP, C_MERGES, C_U_ROWS = range(10)
N_COUNT = 16

EXPORTS = [
    "dartray_grid_create", "dartray_grid_destroy", "dartray_grid_info", "dartray_nside_sca",
    "dartray_s_offset", "dartray_grid_set_rho", "dartray_trace_direct", "dartray_scatter_iter",
    "dartray_trace_adjoint", "dartray_debug_ray_cells", "dartray_workspace_bytes",
    "dartray_last_error", "dartray_version", "dartray_profile_enable", "dartray_profile_read",
    "dartray_set_tuning", "dartray_get_tuning", "dartray_batch_create", "dartray_batch_destroy",
    "dartray_batch_run", "dartray_batch_capture", "dartray_batch_replay", "dartray_trace_direct_noalloc",
    "dartray_observe", "dartray_absorbed", "dartray_dust_emission", "dartray_grid_set_emis",
    "dartray_dust_selfheat",
]


class DartRayError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dartray status {code}: {msg}")
        self.code = code


class GridDesc(C.Structure):
    _fields_ = [
        ("nroot", C.c_int32 * 3),
        ("lo", C.c_double * 3),
        ("root_size", C.c_double),
        ("n_leaves", C.c_int64),
        ("leaf_level", C.POINTER(C.c_int32)),
        ("leaf_ijk", C.POINTER(C.c_int64)),
        ("rho", C.POINTER(C.c_float)),
        ("emis", C.POINTER(C.c_float)),
        ("n_lambda", C.c_int32),
        ("kappa", C.POINTER(C.c_float)),
        ("albedo", C.POINTER(C.c_float)),
        ("g", C.POINTER(C.c_float)),
        ("nside_sca", C.POINTER(C.c_int32)),
        ("n_fwhm", C.c_double),
        ("k_max", C.c_int32),
        ("c_light", C.c_double),
        ("nside_max", C.c_int32),
        ("n_point", C.c_int32),
        ("point_pos", C.POINTER(C.c_double)),
        ("point_lum", C.POINTER(C.c_float)),
    ]


class TraceOpts(C.Structure):
    _fields_ = [
        ("mode", C.c_int32),
        ("adaptive", C.c_int32),
        ("nside", C.c_int32),
        ("nside_max", C.c_int32),
        ("n_rays_min", C.c_double),
        ("f_U", C.c_double),
        ("a_RT", C.c_double),
        ("r_pre", C.c_double),
        ("frame", C.c_double * 9),
        ("source_mask", C.c_void_p),
        ("flags", C.c_uint32),
        ("max_steps", C.c_int64),
        ("n_rays_max", C.c_double),
    ]


class FieldsC(C.Structure):
    _fields_ = [
        ("U", C.c_void_p),
        ("U_LL", C.c_void_p),
        ("U_pass", C.c_void_p),
        ("S_total", C.c_void_p),
        ("S_pending", C.c_void_p),
        ("S_next", C.c_void_p),
        ("tally", C.c_void_p),
        ("counters", C.c_void_p),
        ("escape", C.c_void_p),
    ]


OBS_DISTANT, OBS_INTERNAL = 0, 1


class Observer(C.Structure):
    """dartray_observer: a distant observer (image plane) or an internal one
    (HEALPix all-sky map)."""
    _fields_ = [
        ("kind", C.c_int32),
        ("dir", C.c_double * 3),
        ("up", C.c_double * 3),
        ("centre", C.c_double * 3),
        ("pixel_size", C.c_double),
        ("nx", C.c_int32),
        ("ny", C.c_int32),
        ("pos", C.c_double * 3),
        ("nside_map", C.c_int32),
        ("frame", C.c_double * 9),
    ]


def observer(kind, dir=(0, 0, 1), up=(0, 1, 0), centre=(0, 0, 0), pixel_size=1.0, nx=1, ny=1, pos=(0, 0, 0),
             nside_map=1, frame=None) -> Observer:
    o = Observer()
    o.kind = OBS_DISTANT if kind == "distant" else OBS_INTERNAL
    o.dir = (C.c_double * 3)(*[float(x) for x in dir])
    o.up = (C.c_double * 3)(*[float(x) for x in up])
    o.centre = (C.c_double * 3)(*[float(x) for x in centre])
    o.pixel_size = float(pixel_size)
    o.nx, o.ny = int(nx), int(ny)
    o.pos = (C.c_double * 3)(*[float(x) for x in pos])
    o.nside_map = int(nside_map)
    fr = np.zeros(9) if frame is None else np.asarray(frame, dtype=np.float64).ravel()
    o.frame = (C.c_double * 9)(*fr.tolist())
    return o


class DustModelC(C.Structure):
    """dartray_dust_model: the equilibrium grain of the emission bands."""
    _fields_ = [
        ("b0", C.c_double),
        ("x0", C.c_double),
        ("t_max", C.c_double),
        ("lam", C.POINTER(C.c_double)),
        ("dlambda", C.POINTER(C.c_double)),
    ]


class SelfHeatOpts(C.Structure):
    _fields_ = [
        ("step1", C.c_int32),
        ("n_scatter", C.c_int32),
        ("max_iter", C.c_int32),
        ("f_L", C.c_double),
        ("conv", C.c_double),
    ]


class Tuning(C.Structure):
    """dartray_tuning: launch parameters of the fixed-ray passes (0 = default);
    item_order also sets the order of the adjoint march's work items."""
    _fields_ = [
        ("lambda_tile", C.c_int32),
        ("block_waves", C.c_int32),
        ("grid_blocks", C.c_int32),
        ("dir_batch", C.c_int32),
        ("item_order", C.c_int32),
    ]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib = None


def load_library():
    """Load libdartray.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1709_03802_amd/build.py "
                           "(or __graft_entry__.build()); there is no fallback path")
    L = C.CDLL(LIB_PATH)
    L.dartray_grid_create.argtypes = [C.POINTER(GridDesc), C.c_void_p, C.POINTER(C.c_void_p)]
    L.dartray_grid_destroy.argtypes = [C.c_void_p]
    L.dartray_grid_info.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
    L.dartray_nside_sca.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]
    L.dartray_s_offset.argtypes = [C.c_void_p, C.c_int32]
    L.dartray_s_offset.restype = C.c_int64
    L.dartray_grid_set_rho.argtypes = [C.c_void_p, C.c_void_p]
    L.dartray_trace_direct.argtypes = [C.c_void_p, C.POINTER(TraceOpts), C.POINTER(FieldsC)]
    L.dartray_trace_direct_noalloc.argtypes = [C.c_void_p, C.POINTER(TraceOpts), C.POINTER(FieldsC)]
    L.dartray_scatter_iter.argtypes = [C.c_void_p, C.POINTER(TraceOpts), C.POINTER(FieldsC), C.POINTER(C.c_double)]
    L.dartray_trace_adjoint.argtypes = [C.c_void_p, C.POINTER(TraceOpts), C.c_int32, C.POINTER(C.c_void_p),
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.dartray_debug_ray_cells.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                          C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                          C.POINTER(C.c_int32)]
    L.dartray_workspace_bytes.argtypes = [C.c_void_p, C.POINTER(TraceOpts), C.POINTER(C.c_size_t)]
    L.dartray_profile_enable.argtypes = [C.c_void_p, C.c_int32]
    L.dartray_profile_read.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.dartray_set_tuning.argtypes = [C.c_void_p, C.POINTER(Tuning)]
    L.dartray_get_tuning.argtypes = [C.c_void_p, C.POINTER(Tuning)]
    L.dartray_batch_create.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p)]
    L.dartray_batch_destroy.argtypes = [C.c_void_p]
    L.dartray_batch_run.argtypes = [C.c_void_p, C.POINTER(TraceOpts), C.POINTER(C.POINTER(FieldsC)), C.c_int32]
    L.dartray_batch_capture.argtypes = [C.c_void_p, C.POINTER(TraceOpts), C.POINTER(C.POINTER(FieldsC)), C.c_int32]
    L.dartray_batch_replay.argtypes = [C.c_void_p]
    L.dartray_observe.argtypes = [C.c_void_p, C.POINTER(Observer), C.c_void_p, C.c_void_p]
    L.dartray_absorbed.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    L.dartray_dust_emission.argtypes = [C.c_void_p, C.POINTER(DustModelC), C.c_void_p, C.c_void_p, C.c_void_p]
    L.dartray_grid_set_emis.argtypes = [C.c_void_p, C.c_void_p]
    L.dartray_dust_selfheat.argtypes = [C.c_void_p, C.POINTER(TraceOpts), C.POINTER(SelfHeatOpts),
                                        C.POINTER(DustModelC), C.c_void_p, C.POINTER(FieldsC), C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                                        C.POINTER(C.c_int32)]
    L.dartray_last_error.restype = C.c_char_p
    L.dartray_version.restype = C.c_char_p
    for name in ("dartray_grid_create", "dartray_grid_destroy", "dartray_grid_info", "dartray_nside_sca",
                 "dartray_grid_set_rho", "dartray_trace_direct", "dartray_trace_direct_noalloc",
                 "dartray_scatter_iter", "dartray_trace_adjoint",
                 "dartray_debug_ray_cells", "dartray_workspace_bytes", "dartray_profile_enable",
                 "dartray_profile_read", "dartray_set_tuning", "dartray_get_tuning", "dartray_batch_create",
                 "dartray_batch_destroy", "dartray_batch_run", "dartray_batch_capture", "dartray_batch_replay",
                 "dartray_observe", "dartray_absorbed", "dartray_dust_emission", "dartray_grid_set_emis",
                 "dartray_dust_selfheat"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(rc):
    if rc != OK:
        msg = load_library().dartray_last_error().decode(errors="replace")
        raise DartRayError(rc, msg)


def version() -> str:
    return load_library().dartray_version().decode()


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


class Grid:
    """Device-side grid built from a ``workloads.Grid``."""

    def __init__(self, grid, stream=None, nside_max=None):
        import torch
        L = load_library()
        self.src = grid
        self.stream = torch.cuda.current_stream() if stream is None else stream
        keep = dict(
            level=np.ascontiguousarray(grid.level, dtype=np.int32),
            ijk=np.ascontiguousarray(grid.ijk, dtype=np.int64),
            rho=np.ascontiguousarray(grid.rho, dtype=np.float32),
            emis=np.ascontiguousarray(grid.emis, dtype=np.float32),
            kappa=np.ascontiguousarray(grid.kappa, dtype=np.float32),
            albedo=np.ascontiguousarray(grid.albedo, dtype=np.float32),
            g=np.ascontiguousarray(grid.g, dtype=np.float32),
            nside_sca=np.ascontiguousarray(grid.nside_sca, dtype=np.int32),
            point_pos=np.ascontiguousarray(getattr(grid, "point_pos", np.zeros((0, 3))), dtype=np.float64),
            point_lum=np.ascontiguousarray(getattr(grid, "point_lum", np.zeros((0, 0))), dtype=np.float32),
        )
        d = GridDesc()
        d.nroot = (C.c_int32 * 3)(*[int(x) for x in grid.nroot])
        d.lo = (C.c_double * 3)(*[float(x) for x in grid.lo])
        d.root_size = float(grid.root_size)
        d.n_leaves = int(grid.n)
        d.leaf_level = _ptr(keep["level"], C.c_int32)
        d.leaf_ijk = _ptr(keep["ijk"], C.c_int64)
        d.rho = _ptr(keep["rho"], C.c_float)
        d.emis = _ptr(keep["emis"], C.c_float)
        d.n_lambda = int(grid.n_lambda)
        d.kappa = _ptr(keep["kappa"], C.c_float)
        d.albedo = _ptr(keep["albedo"], C.c_float)
        d.g = _ptr(keep["g"], C.c_float)
        d.nside_sca = _ptr(keep["nside_sca"], C.c_int32)
        d.n_fwhm = float(grid.n_fwhm)
        d.k_max = int(grid.k_max)
        d.c_light = float(grid.c_light)
        d.nside_max = int(nside_max or 0)
        d.n_point = int(keep["point_pos"].shape[0])
        if d.n_point:
            d.point_pos = _ptr(keep["point_pos"], C.c_double)
            d.point_lum = _ptr(keep["point_lum"], C.c_float)
        h = C.c_void_p()
        _check(L.dartray_grid_create(C.byref(d), C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        n = C.c_int64()
        nl = C.c_int32()
        ss = C.c_int64()
        _check(L.dartray_grid_info(h, C.byref(n), C.byref(nl), C.byref(ss)))
        self.n, self.nl, self.s_size = n.value, nl.value, ss.value
        self.nside_sca = []
        for l in range(self.nl):
            v = C.c_int32()
            _check(L.dartray_nside_sca(h, l, C.byref(v)))
            self.nside_sca.append(v.value)
        self.s_offset = [int(L.dartray_s_offset(h, l)) for l in range(self.nl + 1)]

    def close(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.dartray_grid_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def npix(self, l):
        return 12 * self.nside_sca[l] ** 2

    def workspace_bytes(self, opts: Optional["TraceOpts"] = None) -> int:
        """Device bytes the handle holds, or with opts those a pass with these
        options uses."""
        b = C.c_size_t()
        _check(load_library().dartray_workspace_bytes(self.h, None if opts is None else C.byref(opts), C.byref(b)))
        return b.value

    def profile(self, kinds=PROF_ALL):
        _check(load_library().dartray_profile_enable(self.h, int(kinds)))

    def profile_read(self):
        ms = C.c_double()
        n = C.c_int64()
        _check(load_library().dartray_profile_read(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def set_tuning(self, **kw):
        """Set fixed-ray launch parameters (fields of ``Tuning``; others keep their value)."""
        t = self.tuning()
        for k, v in kw.items():
            if k not in dict(Tuning._fields_):
                raise KeyError(k)
            setattr(t, k, int(v))
        _check(load_library().dartray_set_tuning(self.h, C.byref(t)))

    def tuning(self) -> Tuning:
        t = Tuning()
        _check(load_library().dartray_get_tuning(self.h, C.byref(t)))
        return t

    def set_rho(self, rho_dev):
        _check(load_library().dartray_grid_set_rho(self.h, C.c_void_p(rho_dev.data_ptr())))


class Fields:
    """Caller-owned device buffers (torch tensors) of one run."""

    def __init__(self, grid: Grid, keep_pass_u=False, escape_nside=None):
        """escape_nside: allocate the per-direction escape output of fixed-ray
        passes with that ray Nside."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        f32 = dict(dtype=torch.float32, device=dev)
        self.U = torch.zeros((grid.nl, grid.n), **f32)
        self.U_LL = torch.zeros((grid.nl, grid.n), **f32)
        self.U_pass = torch.zeros((grid.nl, grid.n), **f32) if keep_pass_u else None
        self.S_total = torch.zeros(max(grid.s_size, 1), **f32)
        self.S_pending = torch.zeros(max(grid.s_size, 1), **f32)
        self.S_next = torch.zeros(max(grid.s_size, 1), **f32)
        self.tally = torch.zeros((grid.nl, 8), dtype=torch.float64, device=dev)
        self.counters = torch.zeros(N_COUNT, dtype=torch.int64, device=dev)
        self.escape = (torch.zeros((grid.nl, 12 * escape_nside ** 2), **f32) if escape_nside else None)

    def c(self) -> FieldsC:
        f = FieldsC()
        for name in ("U", "U_LL", "U_pass", "S_total", "S_pending", "S_next", "tally", "counters", "escape"):
            t = getattr(self, name)
            setattr(f, name, None if t is None else t.data_ptr())
        return f


class Batch:
    """Several grids (one stream, one wavelength count) whose fixed-ray passes
    run together: one persistent march launch and one flush launch per
    direction batch for all models; ``capture`` records the whole pass
    sequence as a HIP graph that ``replay`` relaunches."""

    def __init__(self, grids):
        L = load_library()
        self.grids = list(grids)
        arr = (C.c_void_p * len(self.grids))(*[g.h.value for g in self.grids])
        h = C.c_void_p()
        _check(L.dartray_batch_create(arr, len(self.grids), C.byref(h)))
        self.h = h

    def _args(self, policy, fields, frame, counters):
        if len(fields) != len(self.grids):
            raise ValueError("one Fields per grid")
        self._fc = [f.c() for f in fields]
        arr = (C.POINTER(FieldsC) * len(fields))(*[C.pointer(fc) for fc in self._fc])
        return make_opts(policy, MODE_DIRECT, frame, counters=counters), arr

    def run(self, policy, fields, frame=None, counters=True):
        opts, arr = self._args(policy, fields, frame, counters)
        _check(load_library().dartray_batch_run(self.h, C.byref(opts), arr, int(policy.n_scatter)))

    def capture(self, policy, fields, frame=None, counters=True):
        """Record direct pass + policy.n_scatter iterations into fields (kept
        by the caller: the graph writes to these buffers on every replay)."""
        opts, arr = self._args(policy, fields, frame, counters)
        _check(load_library().dartray_batch_capture(self.h, C.byref(opts), arr, int(policy.n_scatter)))

    def replay(self):
        _check(load_library().dartray_batch_replay(self.h))

    def close(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.dartray_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


def make_opts(policy, mode=MODE_DIRECT, frame=None, source_mask=None, counters=True, max_steps=0,
              check=False) -> TraceOpts:
    o = TraceOpts()
    o.mode = mode
    o.adaptive = 1 if policy.adaptive else 0
    o.nside = int(policy.nside)
    o.nside_max = int(policy.nside_max)
    o.n_rays_min = float(policy.n_rays_min)
    o.f_U = float(policy.f_U)
    o.a_RT = float(getattr(policy, "a_RT", 0.0))
    o.r_pre = float(policy.r_pre)
    fr = np.zeros(9) if frame is None else np.asarray(frame, dtype=np.float64).ravel()
    o.frame = (C.c_double * 9)(*fr.tolist())
    o.source_mask = None if source_mask is None else source_mask.data_ptr()
    o.flags = (FLAG_COUNTERS if counters else 0) | (FLAG_CHECK if check else 0) | \
        (FLAG_2D if getattr(policy, "mode_2d", False) else 0)
    o.max_steps = int(max_steps)
    o.n_rays_max = float(getattr(policy, "n_rays_max", 0.0))
    return o


def trace_direct(grid: Grid, opts: TraceOpts, fields: Fields):
    fc = fields.c()
    _check(load_library().dartray_trace_direct(grid.h, C.byref(opts), C.byref(fc)))


def trace_direct_noalloc(grid: Grid, opts: TraceOpts, fields: Fields):
    """The direct pass without any device allocation (fixed rays; work arrays
    in the library's static per-GPU scratch array)."""
    fc = fields.c()
    _check(load_library().dartray_trace_direct_noalloc(grid.h, C.byref(opts), C.byref(fc)))


def scatter_iter(grid: Grid, opts: TraceOpts, fields: Fields, want_rk=True):
    """One scattering iteration; returns r_k (a host synchronisation) or,
    with want_rk=False, None and stays asynchronous."""
    fc = fields.c()
    if not want_rk:
        _check(load_library().dartray_scatter_iter(grid.h, C.byref(opts), C.byref(fc), None))
        return None
    rk = C.c_double()
    _check(load_library().dartray_scatter_iter(grid.h, C.byref(opts), C.byref(fc), C.byref(rk)))
    return rk.value


def trace_adjoint(grid: Grid, opts: TraceOpts, S_hist, dJ_dU, dJ_drho, dJ_desc=None, dJ_dS=None):
    """dJ/drho into dJ_drho (device float [n]) for dJ_dU (device [nl, n] or
    None), dJ_dS (device, S layout, or None: the derivative with respect to
    S_total, the scattered luminosity of every order) and dJ_desc (device
    [nl, 12 nside^2] or None: the derivative with respect to the escaping
    luminosity summed over the passes).

    S_hist: the S_pending tensors each scattering iteration of the forward run
    processed, in order (``DartRayFn`` keeps them)."""
    arr = (C.c_void_p * max(len(S_hist), 1))(*[t.data_ptr() for t in S_hist])
    _check(load_library().dartray_trace_adjoint(grid.h, C.byref(opts), len(S_hist), arr,
                                                None if dJ_dU is None else C.c_void_p(dJ_dU.data_ptr()),
                                                None if dJ_dS is None else C.c_void_p(dJ_dS.data_ptr()),
                                                None if dJ_desc is None else C.c_void_p(dJ_desc.data_ptr()),
                                                C.c_void_p(dJ_drho.data_ptr())))


def _autograd():
    import torch

    class DartRayFn(torch.autograd.Function):
        """rho (device float [n]) -> (U [n_lambda, n], F [n_lambda, 12 nside^2],
        S_total [s_size]) for a fixed-ray run (direct pass + policy.n_scatter
        scattering iterations), F being the escaping luminosity by direction
        summed over the passes and S_total the scattered luminosity of every
        order (j_sca = S_total / (V 4 pi / N_pix)); backward by the adjoint
        march."""

        @staticmethod
        def forward(ctx, rho, grid, policy, frame=None):
            # outputs the loss does not use get no gradient (None, not a
            # zero tensor), so the adjoint skips their terms: an all-zero
            # dJ/dS_total would still gather the scattered-light gradient
            # for the last scattering pass
            ctx.set_materialize_grads(False)
            grid.set_rho(rho.detach().contiguous())
            f = Fields(grid, escape_nside=policy.nside)
            opts = make_opts(policy, MODE_DIRECT, frame, counters=False)
            trace_direct(grid, opts, f)
            F = f.escape.clone()
            hist = []
            for _ in range(policy.n_scatter):
                hist.append(f.S_pending.clone())
                scatter_iter(grid, opts, f, want_rk=False)
                F += f.escape
            ctx.grid, ctx.opts, ctx.hist = grid, opts, hist
            ctx.save_for_backward(rho)
            return f.U.clone(), F, f.S_total[:grid.s_size].clone()

        @staticmethod
        def backward(ctx, gU, gF, gS):
            (rho,) = ctx.saved_tensors
            ctx.grid.set_rho(rho.detach().contiguous())
            drho = torch.empty_like(rho)
            gU = None if gU is None else gU.contiguous().to(torch.float32)
            gF = None if gF is None else gF.contiguous().to(torch.float32)
            gS = None if gS is None else gS.contiguous().to(torch.float32)
            trace_adjoint(ctx.grid, ctx.opts, ctx.hist, gU, drho, dJ_desc=gF, dJ_dS=gS)
            return drho, None, None, None

    return DartRayFn


_fn = None


def rfed_full(rho, grid: Grid, policy, frame=None):
    """Differentiable (U(rho), F(rho), S_total(rho)): energy density, escaping
    luminosity by direction and scattered luminosity of every order (see
    ``DartRayFn``)."""
    global _fn
    if _fn is None:
        _fn = _autograd()
    return _fn.apply(rho, grid, policy, frame)


def rfed_escape(rho, grid: Grid, policy, frame=None):
    """Differentiable (U(rho), F(rho)): energy density and escaping luminosity
    by direction (see ``DartRayFn``)."""
    return rfed_full(rho, grid, policy, frame)[:2]


def rfed(rho, grid: Grid, policy, frame=None):
    """Differentiable energy density U(rho)."""
    return rfed_escape(rho, grid, policy, frame)[0]


def observe(grid: Grid, obs: Observer, S_total=None):
    """Observer map (device double [n_lambda, npix]) of the grid's emission and,
    when S_total (device float, S layout) is given, its scattered light."""
    import torch
    npix = obs.nx * obs.ny if obs.kind == OBS_DISTANT else 12 * obs.nside_map ** 2
    out = torch.empty((grid.nl, npix), dtype=torch.float64, device=torch.device("cuda", torch.cuda.current_device()))
    _check(load_library().dartray_observe(grid.h, C.byref(obs), None if S_total is None else C.c_void_p(S_total.data_ptr()),
                                          C.c_void_p(out.data_ptr())))
    return out


def debug_ray_cells(grid: Grid, origins, dirs, max_cross=4096):
    o = np.ascontiguousarray(origins, dtype=np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    nr = o.shape[0]
    cells = np.zeros((nr, max_cross), dtype=np.int64)
    lens = np.zeros((nr, max_cross), dtype=np.float64)
    counts = np.zeros(nr, dtype=np.int32)
    _check(load_library().dartray_debug_ray_cells(grid.h, nr, _ptr(o, C.c_double), _ptr(d, C.c_double), max_cross,
                                                  _ptr(cells, C.c_int64), _ptr(lens, C.c_double),
                                                  _ptr(counts, C.c_int32)))
    return [(cells[i, :counts[i]], lens[i, :counts[i]]) for i in range(nr)]


@dataclass
class RunOutput:
    fields: Fields
    tallies: list            # per pass, numpy [nl, 8]
    counters: list           # per pass, numpy [8]
    r_k: list
    escape: list = field(default_factory=list)   # per pass after step 1, [nl, 12 nside^2] (fixed rays)


def run(grid: Grid, policy, frame=None, source_mask=None, fields: Optional[Fields] = None,
        collect=True, passes=None, escape=False) -> RunOutput:
    """Step 1 (adaptive + step1), direct pass, scattering iterations (at most
    policy.n_scatter; with policy.f_L > 0 they stop once r_k < f_L).  With
    ``escape`` (fixed rays) the new Fields carry the per-direction escape."""
    if fields is None:
        f = Fields(grid, escape_nside=policy.nside if escape and not policy.adaptive else None)
    else:
        f = fields
    tallies, counters, rks, escapes = [], [], [], []
    if policy.adaptive and policy.step1:
        trace_direct(grid, make_opts(policy, MODE_STEP1, frame, source_mask), f)
        if collect:
            tallies.append(f.tally.cpu().numpy().copy())
            counters.append(f.counters.cpu().numpy().copy())
    n_pass = 1 + policy.n_scatter if passes is None else passes
    f_L = float(getattr(policy, "f_L", 0.0))
    for k in range(n_pass):
        if k == 0:
            trace_direct(grid, make_opts(policy, MODE_DIRECT, frame, source_mask), f)
        else:
            rk = scatter_iter(grid, make_opts(policy, MODE_DIRECT, frame), f, want_rk=collect or f_L > 0.0)
            if rk is not None:
                rks.append(rk)
        if collect:
            tallies.append(f.tally.cpu().numpy().copy())
            counters.append(f.counters.cpu().numpy().copy())
            if f.escape is not None and not policy.adaptive:
                escapes.append(f.escape.cpu().numpy().copy())
        if k > 0 and f_L > 0.0 and rks[-1] < f_L:
            break   # convergence test of the scattering iterations (Sect. 2)
    return RunOutput(f, tallies, counters, rks, escapes)


# ---------------------------------------------------------------------------
# Dust emission and the self-heating loop (Sect. 3.3)
# ---------------------------------------------------------------------------


def _dust_c(dust):
    lam = np.ascontiguousarray(dust.lambdas_um, dtype=np.float64)
    dl = np.ascontiguousarray(dust.dlambda_um, dtype=np.float64)
    d = DustModelC(float(dust.b0), float(dust.x0), float(dust.t_max), _ptr(lam, C.c_double), _ptr(dl, C.c_double))
    return d, (lam, dl)


def absorbed(grid: Grid, U, A=None):
    """A (device double [n]) += the luminosity the dust of each cell absorbs
    from the energy density U (device float [n_lambda, n])."""
    import torch
    if A is None:
        A = torch.zeros(grid.n, dtype=torch.float64, device=U.device)
    _check(load_library().dartray_absorbed(grid.h, C.c_void_p(U.data_ptr()), C.c_void_p(A.data_ptr())))
    return A


def dust_emission(grid: Grid, dust, A):
    """Equilibrium temperature [n] and band emission [n_lambda, n] (device
    double) of the emitting grid's cells for absorbed luminosities A."""
    import torch
    T = torch.empty(grid.n, dtype=torch.float64, device=A.device)
    j = torch.empty((grid.nl, grid.n), dtype=torch.float64, device=A.device)
    d, keep = _dust_c(dust)
    _check(load_library().dartray_dust_emission(grid.h, C.byref(d), C.c_void_p(A.data_ptr()),
                                                C.c_void_p(T.data_ptr()), C.c_void_p(j.data_ptr())))
    return T, j


def set_emis(grid: Grid, j):
    """Replace the grid's emission (device double [n_lambda, n])."""
    _check(load_library().dartray_grid_set_emis(grid.h, C.c_void_p(j.data_ptr())))


@dataclass
class SelfHeatOutput:
    T: object              # device double [n]
    j: object              # device double [nl, n], the converged emission
    j_traced: object       # device double [nl, n], the emission whose light U holds
    fields: Fields         # U, S_total of the dust emission
    ratios: list           # max dj / j_prev after each dust RT calculation
    A_star: object         # device double [n]


def dust_selfheat(star_grid: Grid, U_star, dust_grid: Grid, policy, dust, frame=None, fields=None) -> SelfHeatOutput:
    """Absorbed stellar luminosity from U_star (device float, the stellar
    grid's U), then the self-heating loop on the dust grid."""
    import torch
    dev = U_star.device
    A_star = absorbed(star_grid, U_star)
    f = Fields(dust_grid) if fields is None else fields
    n, nl = dust_grid.n, dust_grid.nl
    T = torch.zeros(n, dtype=torch.float64, device=dev)
    j = torch.zeros((nl, n), dtype=torch.float64, device=dev)
    jt = torch.zeros((nl, n), dtype=torch.float64, device=dev)
    work = torch.zeros(n * (1 + nl), dtype=torch.float64, device=dev)
    so = SelfHeatOpts(int(bool(policy.adaptive and policy.step1)), int(policy.n_scatter), int(dust.max_iter),
                      float(getattr(policy, "f_L", 0.0)), float(dust.conv))
    d, keep = _dust_c(dust)
    ratios = (C.c_double * int(dust.max_iter))()
    n_rt = C.c_int32(0)
    o = make_opts(policy, MODE_DIRECT, frame)
    fc = f.c()
    _check(load_library().dartray_dust_selfheat(dust_grid.h, C.byref(o), C.byref(so), C.byref(d),
                                                C.c_void_p(A_star.data_ptr()), C.byref(fc), C.c_void_p(T.data_ptr()),
                                                C.c_void_p(j.data_ptr()), C.c_void_p(jt.data_ptr()),
                                                C.c_void_p(work.data_ptr()), ratios, C.byref(n_rt)))
    return SelfHeatOutput(T, j, jt, f, [ratios[i] for i in range(n_rt.value)], A_star)

"""FP64 CPU oracle for the DART-Ray ray-march (test infrastructure).

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may import this package.  The product path never does: it runs on the GPU
library alone.  The C source is ``dartray_oracle.c``; ``build()`` compiles it
with gcc into ``liboracle.so`` next to it.

Python-side helpers here only marshal arrays and chain passes in the order of
the paper's algorithm (Sect. 2: step 1, direct light, scattering iterations
until the f_L test or the iteration limit), and chain the adjoint passes in
reverse order.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dartray_oracle.c")
# DARTRAY_ORACLE_LIB names a prebuilt oracle library to load instead (the
# sanitizer run of sanitize.sh); it is then not rebuilt here
LIB_OVERRIDE = os.environ.get("DARTRAY_ORACLE_LIB")
LIB = LIB_OVERRIDE or os.path.join(HERE, "liboracle.so")

STEP1, DIRECT, SCATTER = 0, 1, 2
T_EMITTED, T_ABSORBED, T_SCATTERED, T_ESCAPED, T_CUT, T_SKIPPED = range(6)
C_CROSS, C_RAYS, C_SPLITS, C_CUTS, C_ESCAPES, C_DEPOSITS, C_SKIPS, C_MAXSTEP, C_MERGES = range(9)


def build(force: bool = False) -> str:
    """Compile the oracle (plain C, FP64, OpenMP).  No contraction into fused
    multiply-adds: each FP64 step rounds on its own, which is the rule that
    decides a value lying on a pixel or cell edge."""
    if LIB_OVERRIDE:
        return LIB
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class GridDesc(C.Structure):
    _fields_ = [
        ("nroot", C.c_int32 * 3),
        ("lo", C.c_double * 3),
        ("root_size", C.c_double),
        ("n_leaves", C.c_int64),
        ("level", C.POINTER(C.c_int32)),
        ("ijk", C.POINTER(C.c_int64)),
        ("rho", C.POINTER(C.c_double)),
        ("emis", C.POINTER(C.c_double)),
        ("n_lambda", C.c_int32),
        ("kappa", C.POINTER(C.c_double)),
        ("albedo", C.POINTER(C.c_double)),
        ("g", C.POINTER(C.c_double)),
        ("nside_sca", C.POINTER(C.c_int32)),
        ("n_fwhm", C.c_double),
        ("k_max", C.c_int32),
        ("c_light", C.c_double),
        ("n_point", C.c_int64),
        ("point_pos", C.POINTER(C.c_double)),
        ("point_lum", C.POINTER(C.c_double)),
    ]


class PassOpts(C.Structure):
    _fields_ = [
        ("mode", C.c_int32),
        ("adaptive", C.c_int32),
        ("nside", C.c_int32),
        ("nside_max", C.c_int32),
        ("n_rays_min", C.c_double),
        ("f_U", C.c_double),
        ("r_pre", C.c_double),
        ("frame", C.c_double * 9),
        ("source_mask", C.POINTER(C.c_uint8)),
        ("max_steps", C.c_int64),
        ("n_threads", C.c_int32),
        ("a_RT", C.c_double),
        ("mode_2d", C.c_int32),
        ("n_rays_max", C.c_double),
    ]


class Observer(C.Structure):
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


_lib = None


class DustModelC(C.Structure):
    _fields_ = [
        ("b0", C.c_double),
        ("x0", C.c_double),
        ("t_max", C.c_double),
        ("lam", C.POINTER(C.c_double)),
        ("dlambda", C.POINTER(C.c_double)),
    ]


def lib():
    global _lib
    if _lib is None:
        path = build()
        L = C.CDLL(path)
        L.orc_healpix_vec.argtypes = [C.c_int64, C.c_int64, C.POINTER(C.c_double)]
        L.orc_hg.argtypes = [C.c_double, C.c_double]
        L.orc_hg.restype = C.c_double
        L.orc_hg_fwhm.argtypes = [C.c_double]
        L.orc_hg_fwhm.restype = C.c_double
        L.orc_k_hp_real.argtypes = [C.c_double, C.c_double]
        L.orc_k_hp_real.restype = C.c_double
        L.orc_k_hp.argtypes = [C.c_double, C.c_double, C.c_int]
        L.orc_k_hp.restype = C.c_int
        L.orc_hg_weights.argtypes = [C.c_int, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]
        L.orc_model_create.argtypes = [C.POINTER(GridDesc), C.POINTER(C.c_void_p)]
        L.orc_model_create.restype = C.c_int
        L.orc_model_destroy.argtypes = [C.c_void_p]
        L.orc_model_s_size.argtypes = [C.c_void_p]
        L.orc_model_s_size.restype = C.c_int64
        L.orc_model_nside_sca.argtypes = [C.c_void_p, C.c_int]
        L.orc_model_nside_sca.restype = C.c_int32
        L.orc_model_s_offset.argtypes = [C.c_void_p, C.c_int]
        L.orc_model_s_offset.restype = C.c_int64
        L.orc_locate.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_locate.restype = C.c_int64
        L.orc_trace_cells.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_double,
                                      C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double)]
        L.orc_trace_cells.restype = C.c_int64
        L.orc_crossings.argtypes = L.orc_trace_cells.argtypes
        L.orc_crossings.restype = C.c_int64
        L.orc_is_graze.argtypes = [C.c_double, C.c_double]
        L.orc_is_graze.restype = C.c_int
        L.orc_count_sources.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_double)]
        L.orc_count_sources.restype = C.c_int64
        L.orc_run_pass.argtypes = [C.c_void_p, C.POINTER(PassOpts), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.orc_run_pass.restype = C.c_int
        L.orc_adjoint_pass.argtypes = [C.c_void_p, C.POINTER(PassOpts), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.POINTER(C.c_double)]
        L.orc_adjoint_pass.restype = C.c_int
        L.orc_healpix_pix.argtypes = [C.c_int64, C.POINTER(C.c_double)]
        L.orc_healpix_pix.restype = C.c_int64
        L.orc_observe.argtypes = [C.c_void_p, C.POINTER(Observer), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_observe.restype = C.c_int
        L.orc_absorbed.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_dust_power.argtypes = [C.c_void_p, C.POINTER(DustModelC), C.c_double]
        L.orc_dust_power.restype = C.c_double
        L.orc_dust_emission.argtypes = [C.c_void_p, C.POINTER(DustModelC), C.POINTER(C.c_double),
                                        C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_dust_emission.restype = C.c_int
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _dvec(v):
    return (C.c_double * 3)(*[float(x) for x in v])


# ---------------------------------------------------------------------------
# Geometry helpers
# ---------------------------------------------------------------------------


def healpix_vec(nside: int, pix: int) -> np.ndarray:
    out = (C.c_double * 3)()
    lib().orc_healpix_vec(nside, pix, out)
    return np.array(out[:])


def healpix_vecs(nside: int) -> np.ndarray:
    return np.array([healpix_vec(nside, p) for p in range(12 * nside * nside)])


def healpix_pix(nside: int, v) -> int:
    return int(lib().orc_healpix_pix(nside, _dvec(v)))


def observer(kind, dir=(0, 0, 1), up=(0, 1, 0), centre=(0, 0, 0), pixel_size=1.0, nx=1, ny=1, pos=(0, 0, 0),
             nside_map=1, frame=None) -> Observer:
    """kind 'distant' (image of nx x ny pixels of edge pixel_size centred on
    `centre`, seen from direction `dir`) or 'internal' (all-sky HEALPix map at
    nside_map seen from `pos`)."""
    o = Observer()
    o.kind = 0 if kind == "distant" else 1
    o.dir = (C.c_double * 3)(*[float(x) for x in dir])
    o.up = (C.c_double * 3)(*[float(x) for x in up])
    o.centre = (C.c_double * 3)(*[float(x) for x in centre])
    o.pixel_size = float(pixel_size)
    o.nx, o.ny = int(nx), int(ny)
    o.pos = (C.c_double * 3)(*[float(x) for x in pos])
    o.nside_map = int(nside_map)
    fr = np.eye(3) if frame is None else np.asarray(frame, dtype=np.float64)
    o.frame = (C.c_double * 9)(*fr.ravel().tolist())
    return o


def hg(g: float, mu: float) -> float:
    return lib().orc_hg(g, mu)


def hg_fwhm(g: float) -> float:
    return lib().orc_hg_fwhm(g)


def k_hp_real(g: float, n_fwhm: float = 5.0) -> float:
    return lib().orc_k_hp_real(g, n_fwhm)


def k_hp(g: float, n_fwhm: float = 5.0, k_max: int = 2) -> int:
    return lib().orc_k_hp(g, n_fwhm, k_max)


def hg_weights(nside_sca: int, g: float, n, frame=None) -> np.ndarray:
    frame = np.eye(3) if frame is None else np.asarray(frame, dtype=np.float64)
    w = np.zeros(12 * nside_sca * nside_sca)
    fr = np.ascontiguousarray(frame, dtype=np.float64).ravel()
    nn = np.ascontiguousarray(n, dtype=np.float64)
    lib().orc_hg_weights(nside_sca, g, _p(nn, C.c_double), _p(fr, C.c_double), _p(w, C.c_double))
    return w


class Model:
    """Oracle view of a workload grid (keeps the numpy arrays alive)."""

    def __init__(self, grid):
        self.grid = grid
        self._keep = dict(
            level=np.ascontiguousarray(grid.level, dtype=np.int32),
            ijk=np.ascontiguousarray(grid.ijk, dtype=np.int64),
            rho=np.ascontiguousarray(grid.rho, dtype=np.float64),
            emis=np.ascontiguousarray(grid.emis, dtype=np.float64),
            kappa=np.ascontiguousarray(grid.kappa, dtype=np.float64),
            albedo=np.ascontiguousarray(grid.albedo, dtype=np.float64),
            g=np.ascontiguousarray(grid.g, dtype=np.float64),
            nside_sca=np.ascontiguousarray(grid.nside_sca, dtype=np.int32),
            point_pos=np.ascontiguousarray(getattr(grid, "point_pos", np.zeros((0, 3))), dtype=np.float64),
            point_lum=np.ascontiguousarray(getattr(grid, "point_lum", np.zeros((0, 0))), dtype=np.float64),
        )
        k = self._keep
        d = GridDesc()
        d.nroot = (C.c_int32 * 3)(*[int(x) for x in grid.nroot])
        d.lo = (C.c_double * 3)(*[float(x) for x in grid.lo])
        d.root_size = float(grid.root_size)
        d.n_leaves = grid.n
        d.level = _p(k["level"], C.c_int32)
        d.ijk = _p(k["ijk"], C.c_int64)
        d.rho = _p(k["rho"], C.c_double)
        d.emis = _p(k["emis"], C.c_double)
        d.n_lambda = grid.n_lambda
        d.kappa = _p(k["kappa"], C.c_double)
        d.albedo = _p(k["albedo"], C.c_double)
        d.g = _p(k["g"], C.c_double)
        d.nside_sca = _p(k["nside_sca"], C.c_int32)
        d.n_fwhm = float(grid.n_fwhm)
        d.k_max = int(grid.k_max)
        d.c_light = float(grid.c_light)
        d.n_point = int(k["point_pos"].shape[0])
        if d.n_point:
            d.point_pos = _p(k["point_pos"], C.c_double)
            d.point_lum = _p(k["point_lum"], C.c_double)
        self._desc = d
        h = C.c_void_p()
        rc = lib().orc_model_create(C.byref(d), C.byref(h))
        if rc != 0:
            raise ValueError(f"oracle rejected the grid (status {rc})")
        self.h = h
        self.n = grid.n
        self.nl = grid.n_lambda
        self.s_size = lib().orc_model_s_size(h)
        self.nside_sca = [lib().orc_model_nside_sca(h, l) for l in range(self.nl)]
        self.s_offset = [lib().orc_model_s_offset(h, l) for l in range(self.nl + 1)]

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.orc_model_destroy(self.h)
            self.h = None

    def npix(self, l):
        return 12 * self.nside_sca[l] ** 2

    def s_block(self, S, l):
        """View of wavelength block l of an S array as [n, npix]."""
        return S[self.s_offset[l]:self.s_offset[l + 1]].reshape(self.n, self.npix(l))

    def locate(self, p, d):
        return int(lib().orc_locate(self.h, _dvec(p), _dvec(d)))

    def trace_cells(self, o, d, t0=0.0, max_cross=100000):
        cells = np.zeros(max_cross, dtype=np.int64)
        lens = np.zeros(max_cross)
        tin = np.zeros(max_cross)
        n = lib().orc_trace_cells(self.h, _dvec(o), _dvec(d), float(t0), max_cross,
                                  _p(cells, C.c_int64), _p(lens, C.c_double), _p(tin, C.c_double))
        return cells[:n], lens[:n], tin[:n]

    def crossings(self, o, d, t0=0.0, max_cross=100000):
        """Crossings of positive length as a pass walks them (grazes folded)."""
        cells = np.zeros(max_cross, dtype=np.int64)
        lens = np.zeros(max_cross)
        tin = np.zeros(max_cross)
        n = lib().orc_crossings(self.h, _dvec(o), _dvec(d), float(t0), max_cross,
                                _p(cells, C.c_int64), _p(lens, C.c_double), _p(tin, C.c_double))
        return cells[:n], lens[:n], tin[:n]

    def count_sources(self, mode, S_pending=None):
        Sp = None if S_pending is None else np.ascontiguousarray(S_pending, dtype=np.float64)
        return int(lib().orc_count_sources(self.h, mode, None if Sp is None else _p(Sp, C.c_double)))

    def observe(self, obs: Observer, S_total=None) -> np.ndarray:
        """Observer map [n_lambda, npix]: surface brightness of every cell's
        emission (and scattered light from S_total) attenuated to the observer."""
        npix = obs.nx * obs.ny if obs.kind == 0 else 12 * obs.nside_map ** 2
        out = np.zeros(self.nl * npix)
        St = None if S_total is None else np.ascontiguousarray(S_total, dtype=np.float64)
        rc = lib().orc_observe(self.h, C.byref(obs), None if St is None else _p(St, C.c_double), _p(out, C.c_double))
        if rc != 0:
            raise ValueError(f"oracle observe failed (status {rc})")
        return out.reshape(self.nl, npix)

    def run_pass(self, mode, policy, S_pending=None, U_LL=None, frame=None, source_mask=None,
                 max_steps=0, n_threads=0):
        o, mask = _opts(mode, policy, frame, source_mask, n_threads)
        o.max_steps = int(max_steps)
        U_k = np.zeros(self.nl * self.n)
        S_next = np.zeros(max(self.s_size, 1))
        tally = np.zeros(self.nl * 8)
        counters = np.zeros(16, dtype=np.int64)
        nray0 = 12 * int(policy.nside) ** 2
        escape = np.zeros(self.nl * nray0)
        Sp = None if S_pending is None else np.ascontiguousarray(S_pending, dtype=np.float64)
        ULL = None if U_LL is None else np.ascontiguousarray(U_LL, dtype=np.float64).ravel()
        rc = lib().orc_run_pass(self.h, C.byref(o),
                                None if Sp is None else _p(Sp, C.c_double),
                                None if ULL is None else _p(ULL, C.c_double),
                                _p(U_k, C.c_double), _p(S_next, C.c_double), _p(tally, C.c_double),
                                _p(counters, C.c_int64), _p(escape, C.c_double))
        if rc != 0:
            raise ValueError(f"oracle pass failed (status {rc})")
        return PassResult(U_k.reshape(self.nl, self.n), S_next[:self.s_size], tally.reshape(self.nl, 8), counters,
                          escape.reshape(self.nl, nray0))


def _opts(mode, policy, frame=None, source_mask=None, n_threads=0):
    o = PassOpts()
    o.mode = mode
    o.adaptive = 1 if policy.adaptive else 0
    o.nside = int(policy.nside)
    o.nside_max = int(policy.nside_max)
    o.n_rays_min = float(policy.n_rays_min)
    o.f_U = float(policy.f_U)
    o.a_RT = float(getattr(policy, "a_RT", 0.0))
    o.r_pre = float(policy.r_pre)
    fr = np.eye(3) if frame is None else np.asarray(frame, dtype=np.float64)
    o.frame = (C.c_double * 9)(*fr.ravel().tolist())
    keep = None
    if source_mask is not None:
        keep = np.ascontiguousarray(source_mask, dtype=np.uint8)
        o.source_mask = _p(keep, C.c_uint8)
    o.n_threads = int(n_threads)
    o.mode_2d = 1 if getattr(policy, "mode_2d", False) else 0
    o.n_rays_max = float(getattr(policy, "n_rays_max", 0.0))
    return o, keep


def adjoint(model: Model, policy, run_result, Ubar=None, Sbar_last=None, frame=None, source_mask=None, n_threads=0,
            Ebar=None, Sbar_total=None):
    """dJ/drho for a loss J(U, S_total, F) given dJ/dU (and optionally dJ/dS of
    the last, unprocessed order, dJ/dS_total -- S_total = S_1 + ... + S_{K+1},
    so every order receives it -- and dJ/dF for the escaping luminosity F
    summed over the passes, [n_lambda][12 nside^2]), by reverse passes over a
    fixed-ray run."""
    if Ubar is None:
        Ubar = np.zeros((model.nl, model.n))
    Ubar = np.ascontiguousarray(Ubar, dtype=np.float64).reshape(model.nl, model.n)
    Eb = None if Ebar is None else np.ascontiguousarray(Ebar, dtype=np.float64).reshape(model.nl, -1)
    rho_bar = np.zeros(model.n)
    passes = [r for r in run_result.passes]
    pend = [None] + [passes[k - 1].S for k in range(1, len(passes))]   # emission of pass k
    St = None if Sbar_total is None else np.ascontiguousarray(Sbar_total, dtype=np.float64)

    def plus(a, b):
        if a is None:
            return b
        return a if b is None else np.ascontiguousarray(a + b)

    Sbar = plus(None if Sbar_last is None else np.ascontiguousarray(Sbar_last, dtype=np.float64), St)
    for k in range(len(passes) - 1, -1, -1):
        mode = DIRECT if k == 0 else SCATTER
        o, keep = _opts(mode, policy, frame, source_mask if k == 0 else None, n_threads)
        Sbar_k = np.zeros(max(model.s_size, 1))
        Sp = None if pend[k] is None else np.ascontiguousarray(pend[k], dtype=np.float64)
        rc = lib().orc_adjoint_pass(model.h, C.byref(o), None if Sp is None else _p(Sp, C.c_double),
                                    _p(Ubar, C.c_double), None if Sbar is None else _p(Sbar, C.c_double),
                                    None if Eb is None else _p(Eb, C.c_double),
                                    _p(rho_bar, C.c_double), _p(Sbar_k, C.c_double))
        if rc != 0:
            raise ValueError(f"oracle adjoint failed (status {rc})")
        Sbar = plus(Sbar_k[:model.s_size], St) if k > 0 else None
    return rho_bar


@dataclass
class PassResult:
    U: np.ndarray          # [nl, n]
    S: np.ndarray          # [S size]
    tally: np.ndarray      # [nl, 8]
    counters: np.ndarray   # [16] (C_* slots; the rest zero)
    escape: np.ndarray     # [nl, 12 nside^2] escaping luminosity by launch pixel


@dataclass
class RunResult:
    U: np.ndarray          # total RFED [nl, n]
    U_LL: Optional[np.ndarray]
    S_total: np.ndarray    # all scattering orders, S_1 .. S_{K+1}
    S_pending: np.ndarray  # last, unprocessed order
    passes: list           # PassResult per pass (step 1 first when present)
    escape: np.ndarray     # escaping luminosity summed over the passes after step 1
    r_k: list              # per scattering iteration: sum S_next / sum S after the direct pass


def run(model: Model, policy, frame=None, source_mask=None, n_threads=0, U_LL_init=None,
        passes=None, U_init=None, S_init=None) -> RunResult:
    """Step 1 (optional), the direct pass and the scattering iterations (Sect. 2).

    U_LL is the step-1 result, then the running U after every pass (the
    footnote of Sect. 2).  ``U_LL_init`` replaces step 1 by a given U_LL.
    ``passes`` limits the number of passes after step 1 (direct counts as 1).
    ``U_init`` / ``S_init`` start the running U and S_total from given values
    (a dust self-heating iteration continues the previous one's, Sect. 3.3).
    With policy.f_L > 0 the iterations stop once the pending scattered
    luminosity falls below f_L times the total scattered in the direct pass.
    """
    results = []
    U_LL = None
    if policy.adaptive:
        if U_LL_init is not None:
            U_LL = np.array(U_LL_init, dtype=np.float64).reshape(model.nl, model.n)
        elif policy.step1:
            r = model.run_pass(STEP1, policy, frame=frame, source_mask=source_mask, n_threads=n_threads)
            results.append(r)
            U_LL = r.U.copy()
        else:
            U_LL = np.zeros((model.nl, model.n))
    n_pass = 1 + policy.n_scatter if passes is None else passes
    f_L = float(getattr(policy, "f_L", 0.0))
    r_k = []
    U = np.zeros((model.nl, model.n)) if U_init is None else \
        np.array(U_init, dtype=np.float64).reshape(model.nl, model.n)
    S_total = np.zeros(model.s_size) if S_init is None else np.array(S_init, dtype=np.float64).reshape(model.s_size)
    S_pending = None
    escape = np.zeros((model.nl, 12 * int(policy.nside) ** 2))
    for k in range(n_pass):
        mode = DIRECT if k == 0 else SCATTER
        r = model.run_pass(mode, policy, S_pending=S_pending, U_LL=U_LL, frame=frame,
                           source_mask=source_mask if k == 0 else None, n_threads=n_threads)
        results.append(r)
        U += r.U
        S_total += r.S
        S_pending = r.S
        escape += r.escape
        if policy.adaptive:
            U_LL = U.copy()
        if k == 0:
            s1 = float(np.sum(r.S))
        else:
            # pending scattered luminosity over the total scattered in the direct pass
            r_k.append(float(np.sum(r.S)) / s1 if s1 > 0.0 else 0.0)
            if f_L > 0.0 and r_k[-1] < f_L:
                break
    return RunResult(U=U, U_LL=U_LL, S_total=S_total, S_pending=S_pending, passes=results, escape=escape,
                     r_k=r_k)


# ---------------------------------------------------------------------------
# Dust emission and the self-heating loop (Sect. 3.3)
# ---------------------------------------------------------------------------


def _dust_c(dust):
    lam = np.ascontiguousarray(dust.lambdas_um, dtype=np.float64)
    dl = np.ascontiguousarray(dust.dlambda_um, dtype=np.float64)
    d = DustModelC(float(dust.b0), float(dust.x0), float(dust.t_max), _p(lam, C.c_double), _p(dl, C.c_double))
    return d, (lam, dl)


def absorbed(model: Model, U) -> np.ndarray:
    """Luminosity absorbed by the dust of each cell, summed over the grid's
    bands: (1 - albedo) kappa rho V c U."""
    A = np.zeros(model.n)
    Uc = np.ascontiguousarray(U, dtype=np.float64).reshape(model.nl, model.n)
    lib().orc_absorbed(model.h, _p(Uc, C.c_double), _p(A, C.c_double))
    return A


def dust_power(model: Model, dust, T: float) -> float:
    """Power a unit dust mass emits over the model's bands at temperature T."""
    d, keep = _dust_c(dust)
    return float(lib().orc_dust_power(model.h, C.byref(d), float(T)))


def dust_emission(model: Model, dust, A):
    """Equilibrium temperature [n] and band emission j [nl, n] of every cell
    of the emitting grid for absorbed luminosities A [n]."""
    d, keep = _dust_c(dust)
    A = np.ascontiguousarray(A, dtype=np.float64)
    T = np.zeros(model.n)
    j = np.zeros((model.nl, model.n))
    rc = lib().orc_dust_emission(model.h, C.byref(d), _p(A, C.c_double), _p(T, C.c_double), _p(j, C.c_double))
    if rc != 0:
        raise ValueError("dust temperature above t_max")
    return T, j


@dataclass
class SelfHeatResult:
    T: np.ndarray          # [n] temperature of the last emission update
    j: np.ndarray          # [nl, n] emission of the last update (what the grain emits now)
    j_traced: np.ndarray   # [nl, n] emission whose light U and S_total hold
    U: np.ndarray          # [nl, n] dust-emission RFED
    S_total: np.ndarray    # dust-emission scattered luminosity
    ratios: list           # per update after the first RT: max dj / j_prev
    runs: list             # RunResult of every dust RT calculation
    A_star: np.ndarray     # [n] absorbed stellar luminosity


def dust_selfheat(star_model: Model, U_star, dust_grid, policy, dust, frame=None, n_threads=0) -> SelfHeatResult:
    """The self-heating procedure of Sect. 3.3, with its own steps in order:

    1. emission from the absorbed stellar luminosity alone;
    2. a dust RT calculation of that emission (step 1 when the policy asks,
       the direct pass, the scattering iterations);
    3. the emission recomputed from the absorbed stellar plus dust light;
    4. dj = j - j_prev;
    5. a dust RT calculation of dj alone, with U_LL, U and S_total starting
       from the previous iteration's U and S_total (no step 1);
    6. steps 3-5 repeated until dj / j_prev < dust.conv at every cell and band.

    dj is not negative in exact arithmetic (more absorbed light, a warmer
    grain, more emission in every band); rounding residues below zero are
    dropped.  The loop ends after step 4 once converged, so the returned j is
    the converged emission and j_traced the emission whose light was traced;
    a cell or band with j_prev = 0 < dj is not converged.
    """
    A_star = absorbed(star_model, U_star)
    base = Model(dust_grid)
    T, j = dust_emission(base, dust, A_star)
    j_prev = np.zeros_like(j)
    dj = j.copy()
    U = None
    S = None
    ratios, runs = [], []
    for it in range(int(dust.max_iter)):
        g = dust_grid.copy()
        g.emis = dj
        r = run(Model(g), policy, frame=frame, n_threads=n_threads, U_init=U, S_init=S,
                U_LL_init=U if (it > 0 and policy.adaptive) else None)
        runs.append(r)
        U, S = r.U, r.S_total
        j_prev = j_prev + dj
        T, j = dust_emission(base, dust, A_star + absorbed(base, U))
        dj = np.maximum(j - j_prev, 0.0)
        with np.errstate(divide="ignore", invalid="ignore"):
            q = np.where(j_prev > 0.0, dj / np.where(j_prev > 0.0, j_prev, 1.0), np.where(dj > 0.0, np.inf, 0.0))
        ratios.append(float(q.max()))
        if ratios[-1] < dust.conv:
            break
    return SelfHeatResult(T=T, j=j, j_traced=j_prev, U=U, S_total=S, ratios=ratios, runs=runs, A_star=A_star)

"""Benchmark of the ray-march hot path on one MI355X.

A step is one whole radiative-transfer run of the workload: step 1 (adaptive
rays), the direct-light pass and the scattering iterations, over every
emitting cell, every ray-cell crossing at every wavelength the rays carry.
The metric is ray-cell crossings x wavelengths per second; the numerator is
the device's own crossing counter from the first (untimed) run.

The same invocation checks the GPU against the FP64 oracle (on a seeded
source subset when the oracle cannot run the whole workload in seconds),
checks the FP64 luminosity balance of every pass, times the oracle on the
host cores as the CPU baseline, and measures the dominant march kernel with
HIP events on the library's stream for the roofline figure.

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# random 64-byte atomic rows per second, measured on MI355X with
# paper_1709_03802_amd/ceilings.py (profiles/k_march_adaptive_step1_disk.md):
# rows of 8 FP64 values (the adaptive marches' energy-density rows, footprints
# up to 128 MiB) and rows of 16 FP32 values (the fixed march's direction bins)
ATOMIC_PEAK_ROWS_F64 = 2.35e10
ATOMIC_PEAK_ROWS_F32 = 2.06e10
# scattered single-value atomics, one lane per 64-byte segment
ATOMIC_PEAK_SINGLE = 2.11e10

# HBM bytes per step-1 launch on the disk workload from rocprofv3 FETCH_SIZE /
# WRITE_SIZE (scaled by a plain copy), valid for the kernel sources hashed here
PMC_TRAFFIC = {
    "workload": "disk",
    "bytes_per_launch": 2.6299e+13 + 1.9904e+13,
    "sources_sha256": "608cac3514d632f4c5c1d8321b02dd29be5e62db23aefc70b98a06407b3bc601",
    "profile": "profiles/k_march_adaptive_step1_disk.md",
}
# the same for the adjoint march of the 64^3 clumpy grid at 4 wavelengths, per
# backward step (three launches): HBM bytes, and atomic requests from
# rocprofv3 TCC_ATOMIC (lanes whose cells share a 64-byte segment share one)
PMC_ADJOINT = {
    "workload": "clumpy64",
    "bytes_per_step": 2.0580e+12 + 2.8701e+11,
    "atomic_requests_per_step": 7.4174e+09,
    "sources_sha256": "608cac3514d632f4c5c1d8321b02dd29be5e62db23aefc70b98a06407b3bc601",
    "profile": "profiles/k_march_adjoint_clumpy64_l4.md",
}


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in ("dartray.hip", "dr_internal.h"):
        with open(os.path.join(ROOT, "paper_1709_03802_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def as_f32(grid):
    g = grid.copy()
    for name in ("rho", "emis", "kappa", "albedo", "g"):
        setattr(g, name, getattr(g, name).astype(np.float32).astype(np.float64))
    return g


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def wall(fn, repeats):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(repeats):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / repeats


def run_crossings(out):
    return int(sum(int(c[0]) for c in out.counters))


def batched_lambda(dr, W, repeats=3):
    """32 wavelengths in one march against the per-wavelength forms: the same
    grid with one-wavelength march tiles, and 32 one-wavelength grids."""
    wl = W.by_name("plain16_l32")
    pol = wl.policy
    G = dr.Grid(as_f32(wl.grid))
    f = dr.Fields(G)
    xl = run_crossings(dr.run(G, pol, fields=f)) * wl.grid.n_lambda

    def with_tile(tile):
        def fn():
            G.set_tuning(lambda_tile=tile)
            dr.run(G, pol, fields=f, collect=False)
        return fn

    singles = []
    for lam in wl.grid.lambdas_um:
        g1 = as_f32(W.plain16(lambdas=np.array([lam]), nside=pol.nside, n_scatter=pol.n_scatter).grid)
        G1 = dr.Grid(g1)
        singles.append((G1, dr.Fields(G1)))

    def per_lambda_runs():
        for G1, f1 in singles:
            dr.run(G1, pol, fields=f1, collect=False)

    res = {}
    for name, fn in (("one_march", with_tile(0)), ("tile1", with_tile(1)), ("runs", per_lambda_runs)):
        fn()
        res[name] = wall(fn, repeats)
    G.set_tuning(lambda_tile=0)
    return {"workload": f"{wl.name}: {wl.description}, direct + {pol.n_scatter} scattering",
            "crossings_x_lambda": xl,
            "one_march_ms": 1e3 * res["one_march"], "one_wavelength_tiles_ms": 1e3 * res["tile1"],
            "one_wavelength_runs_ms": 1e3 * res["runs"],
            "value_one_march": xl / res["one_march"], "value_per_wavelength_runs": xl / res["runs"],
            "speedup_vs_tiles": res["tile1"] / res["one_march"], "speedup_vs_runs": res["runs"] / res["one_march"]}


def batched_models(dr, W, repeats=2):
    """Sixteen disk models of uneven size: one after another, as one batch,
    and as a replayed HIP graph of the batch."""
    import torch
    models = W.disk_batch(16)
    pol = models[0].policy
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        Gs = [dr.Grid(as_f32(m.grid), stream=s) for m in models]
        fs = [dr.Fields(G) for G in Gs]
        fg = [dr.Fields(G) for G in Gs]
    torch.cuda.synchronize()
    xl = sum(run_crossings(dr.run(G, pol, fields=f)) for G, f in zip(Gs, fs)) * models[0].grid.n_lambda
    B = dr.Batch(Gs)
    B.capture(pol, fg, counters=False)

    def sequential():
        for G, f in zip(Gs, fs):
            dr.run(G, pol, fields=f, collect=False)

    res = {}
    for name, fn in (("sequential", sequential), ("batch", lambda: B.run(pol, fs, counters=False)),
                     ("graph", B.replay)):
        fn()
        res[name] = wall(fn, repeats)
    B.close()
    return {"workload": f"{len(models)} disk models, {min(m.grid.n for m in models)}..{max(m.grid.n for m in models)} "
                        f"leaves ({sum(m.grid.n for m in models)} total), {models[0].grid.n_lambda} wavelengths, "
                        f"fixed Nside {pol.nside}, direct + {pol.n_scatter} scattering",
            "crossings_x_lambda": xl,
            "sequential_ms": 1e3 * res["sequential"], "batch_ms": 1e3 * res["batch"], "graph_ms": 1e3 * res["graph"],
            "value_graph": xl / res["graph"], "speedup_graph_vs_sequential": res["sequential"] / res["graph"]}


def adjoint_timing(dr, W, repeats=3):
    """Forward run and adjoint march of the four-wavelength 16^3 grid (the
    gradient configuration) and of a 64^3 clumpy grid at 4 wavelengths."""
    import torch
    out = {}
    for name in ("plain16_l4", "clumpy64_l4"):
        wl = W.by_name(name)
        G = dr.Grid(as_f32(wl.grid))
        xl = run_crossings(dr.run(G, wl.policy)) * wl.grid.n_lambda
        rho = torch.tensor(wl.grid.rho, dtype=torch.float32, device="cuda", requires_grad=True)

        def fwd():
            return dr.rfed_escape(rho, G, wl.policy)

        def fwd_bwd():
            U, F = fwd()
            (U.log().sum() + F.log().sum()).backward()

        # the work-item order that suits the grid, as in the --adjoint mode
        order_ms = {}
        for order in (0, 1):
            G.set_tuning(item_order=order)
            fwd_bwd()
            order_ms[order] = 1e3 * wall(fwd_bwd, 1)
        best = min(order_ms, key=order_ms.get)
        G.set_tuning(item_order=best)
        t_f = wall(lambda: fwd(), repeats)
        t_fb = wall(fwd_bwd, repeats)
        out[name] = {"crossings_x_lambda": xl, "forward_ms": 1e3 * t_f, "forward_backward_ms": 1e3 * t_fb,
                     "backward_ms": 1e3 * (t_fb - t_f), "item_order": best,
                     "backward_value": xl / max(t_fb - t_f, 1e-9), "unit": "crossings*lambda/s (adjoint)"}
    return out


def autotuned(dr, W):
    """The autotuner on the 32-wavelength uniform grid (no cache)."""
    from paper_1709_03802_amd import autotune as AT
    wl = W.by_name("plain16_l32")
    G = dr.Grid(as_f32(wl.grid))
    setting, ms, log = AT.tune(G, wl.policy, cache_path=None, rounds=2, repeats=3)
    return {"workload": wl.name, "pass": "scattering iteration", "setting": setting, "tuned_ms": ms,
            "start_ms": log[0][1], "evaluations": len(log)}


def adjoint_bench(args):
    """The gradient configuration: a forward run (direct pass + scattering
    iterations, untimed) and, timed, its adjoint march for dJ/drho with
    J = sum ln U + sum ln F (F the escaping luminosity by direction)."""
    import torch
    from paper_1709_03802_amd import dartray as dr
    from paper_1709_03802_amd import workloads as W

    wl = W.by_name(args.workload)
    pol = wl.policy
    if pol.adaptive:
        print(json.dumps({"error": "the adjoint covers fixed-ray workloads (plain16_l4, clumpy64_l4, plain16, ...)"}))
        sys.exit(2)
    torch.cuda.set_device(0)
    grid = as_f32(wl.grid)
    nl = grid.n_lambda
    G = dr.Grid(grid)
    log(f"adjoint, workload {wl.name}: {wl.description}")
    out = dr.run(G, pol, collect=True)
    torch.cuda.synchronize()
    counters = np.array(out.counters)
    per_pass = [int(c[dr.C_CROSSINGS]) for c in counters]
    crossings = sum(per_pass)
    rho = torch.tensor(grid.rho, dtype=torch.float32, device="cuda", requires_grad=True)

    def forward():
        rho.grad = None
        U, F = dr.rfed_escape(rho, G, pol)
        return U.log().sum() + F.log().sum()

    parity, cpu = None, None
    if not args.no_cpu_baseline and grid.n <= 100_000:
        import oracle
        J = forward()
        J.backward()
        torch.cuda.synchronize()
        g_gpu = rho.grad.cpu().numpy().astype(np.float64)
        m = oracle.Model(grid)
        nthreads = os.cpu_count() or 1
        r = oracle.run(m, pol, n_threads=nthreads)
        t0 = time.perf_counter()
        g_ref = oracle.adjoint(m, pol, r, 1.0 / r.U, Ebar=1.0 / r.escape, n_threads=nthreads)
        t_cpu = time.perf_counter() - t0
        err = float(np.abs(g_gpu - g_ref).max() / np.abs(g_ref).max())
        parity = {"checked": "dJ/drho of the full run against the oracle's adjoint", "max_err_over_max_grad": err,
                  "gate": 1e-4, "pass": bool(err <= 1e-4)}
        cpu = {"value": crossings * nl / t_cpu, "unit": "crossings*lambda/s", "cores": nthreads, "kind": "oracle",
               "sample": f"adjoint of the full {wl.name} run, {crossings} crossings x {nl} wavelengths in {t_cpu:.1f} s"}
        log(f"oracle adjoint in {t_cpu:.1f} s; parity {parity}")

    # the order of work items (tile- or direction-major) that suits the grid:
    # one timed backward of each
    order_ms = {}
    for order in (0, 1):
        G.set_tuning(item_order=order)
        forward().backward()
        J = forward()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        order_ms[order] = 1e3 * (time.perf_counter() - t0)
    best = min(order_ms, key=order_ms.get)
    G.set_tuning(item_order=best)
    log(f"item order: backward ms {order_ms}, using {best}")
    t_f = wall(lambda: forward(), 2)
    for _ in range(args.warmup):
        forward().backward()
    torch.cuda.synchronize()
    G.profile(dr.PROF_ADJOINT)
    t_b = 0.0
    for _ in range(args.steps):
        J = forward()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        t_b += time.perf_counter() - t0
    kern_ms, launches = G.profile_read()
    G.profile(0)
    ms_per_step = 1e3 * t_b / args.steps
    kern_s = 1e-3 * kern_ms / args.steps
    # per crossing, each of the two walks reads the 64-byte leaf record, the
    # dJ/dU row and the scattered-light gradient row (n_lambda FP32 each); the
    # second walk adds the FP64 density gradient of the cell
    per_cross = 2 * (64 + 2 * 4 * nl) + 16
    achieved = crossings * per_cross / kern_s / 1e9
    measured = wl.name == PMC_ADJOINT["workload"] and sources_sha256() == PMC_ADJOINT["sources_sha256"]
    if measured:
        req_rate = PMC_ADJOINT["atomic_requests_per_step"] / kern_s
        atomic_roof = {"achieved": req_rate, "peak": ATOMIC_PEAK_SINGLE, "unit": "atomic requests/s",
                       "frac": req_rate / ATOMIC_PEAK_SINGLE,
                       "requests_per_crossing": PMC_ADJOINT["atomic_requests_per_step"] / crossings}
    else:
        atomic_roof = {"achieved": None, "peak": ATOMIC_PEAK_SINGLE, "unit": "atomic requests/s", "frac": None,
                       "requests_per_crossing": None,
                       "note": "at most one FP64 request per crossing; the count is measured for clumpy64_l4 only"}
    res = {
        "metric": "adjoint ray-cell crossings x lambda per second (1 MI355X), dJ/drho at <= 1e-4 of max |dJ/drho| "
                  "vs the FP64 oracle's adjoint",
        "value": crossings * nl / (t_b / args.steps),
        "unit": "crossings*lambda/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "description": wl.description, "cells": int(grid.n), "n_lambda": nl,
                   "rays": f"fixed nside {pol.nside}", "passes": ["direct"] + [f"scatter{k + 1}" for k in range(pol.n_scatter)],
                   "crossings_per_run": crossings, "crossings_per_pass": per_pass,
                   "step": "backward of one forward run (the forward is run, untimed, before each step)",
                   "forward_ms": 1e3 * t_f, "item_order": best,
                   "backward_ms_by_item_order": {str(k): v for k, v in order_ms.items()},
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": PMC_ADJOINT["bytes_per_step"] / launches * args.steps if measured and launches else None,
                     "kernel": f"k_march_adjoint<{nl_template(nl)}>",
                     "avg_launch_ms": kern_ms / max(launches, 1), "launches_per_step": launches / args.steps,
                     "bytes_per_crossing": per_cross, "crossings_per_step": crossings},
        # the FP64 density-gradient atomics of the second walk against the
        # scattered single-value atomic ceiling
        "atomic_roofline": atomic_roof,
        "cpu_baseline": cpu,
        "parity": parity,
    }
    print(json.dumps(res), flush=True)


def nl_template(k):
    return 1 if k <= 1 else 4 if k <= 4 else 8


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="disk",
                    choices=["disk", "plain16", "plain16_l32", "plain16_l4", "clumpy64_l4", "clumpy128"])
    ap.add_argument("--adjoint", action="store_true",
                    help="time the adjoint march (dJ/drho) of a fixed-ray workload instead of the forward passes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched-wavelength, batched-model and autotuner measurements")
    ap.add_argument("--sample-sources", type=int, default=1536,
                    help="seeded emitting cells whose step 1 (adaptive workloads) is checked against the oracle and "
                         "timed on the CPU (about 12 s of oracle work on 16 cores for the disk); grids too large "
                         "for a whole oracle run use a quarter of them for a direct pass")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1. Sources shard additively "
                                   "across GPUs, but no multi-GPU path exists."}))
        sys.exit(2)
    if args.adjoint:
        adjoint_bench(args)
        return

    import torch
    from paper_1709_03802_amd import dartray as dr
    from paper_1709_03802_amd import workloads as W

    torch.cuda.set_device(0)
    wl = W.by_name(args.workload)
    grid = as_f32(wl.grid)
    pol = wl.policy
    G = dr.Grid(grid, nside_max=max(pol.nside_max, 64))
    f = dr.Fields(G)
    log(f"workload {wl.name}: {wl.description}")

    # ---- first run: counters, balance
    f.U.zero_()
    out = dr.run(G, pol, fields=f, collect=True)
    torch.cuda.synchronize()
    counters = np.array(out.counters)
    crossings = int(counters[:, dr.C_CROSSINGS].sum())
    cross_lambda = crossings * grid.n_lambda
    balance = max(float(np.max(np.abs(t[:, 1:6].sum(axis=1) - t[:, 0]) / np.maximum(t[:, 0], 1e-300)))
                  for t in out.tallies)
    per_pass = [int(c[dr.C_CROSSINGS]) for c in counters]
    log(f"{crossings} crossings per run ({per_pass}), max luminosity-balance residual {balance:.2e}")

    # ---- parity and CPU baseline against the FP64 oracle
    parity, cpu = None, None
    if not args.no_cpu_baseline:
        import oracle
        m = oracle.Model(grid)
        nthreads = os.cpu_count() or 1
        if pol.adaptive:
            rng = np.random.default_rng(1709)
            sample = np.zeros(grid.n, dtype=np.uint8)
            sample[rng.choice(np.flatnonzero(grid.emis.sum(axis=0) > 0), args.sample_sources, replace=False)] = 1
            t0 = time.perf_counter()
            ref = m.run_pass(oracle.STEP1, pol, source_mask=sample, n_threads=nthreads)
            t_cpu = time.perf_counter() - t0
            fs = dr.Fields(G)
            dr.trace_direct(G, dr.make_opts(pol, dr.MODE_STEP1, source_mask=torch.as_tensor(sample).cuda()), fs)
            torch.cuda.synchronize()
            got = fs.U_LL.cpu().numpy().astype(np.float64)
            ref_U = ref.U
            ref_cross = int(ref.counters[oracle.C_CROSS])
            gpu_cross = int(fs.counters.cpu().numpy()[dr.C_CROSSINGS])
            what = f"step 1 of {args.sample_sources} seeded emitting cells"
        elif grid.n > 100_000:
            # too large for the oracle's whole run: the direct pass of seeded
            # star cells over the whole grid
            rng = np.random.default_rng(1709)
            sample = np.zeros(grid.n, dtype=np.uint8)
            sample[rng.choice(np.flatnonzero(grid.emis.sum(axis=0) > 0), args.sample_sources // 4, replace=False)] = 1
            t0 = time.perf_counter()
            ref = m.run_pass(oracle.DIRECT, pol, source_mask=sample, n_threads=nthreads)
            t_cpu = time.perf_counter() - t0
            fs = dr.Fields(G)
            dr.trace_direct(G, dr.make_opts(pol, dr.MODE_DIRECT, source_mask=torch.as_tensor(sample).cuda()), fs)
            torch.cuda.synchronize()
            got = fs.U.cpu().numpy().astype(np.float64)
            ref_U = ref.U
            ref_cross = int(ref.counters[oracle.C_CROSS])
            gpu_cross = int(fs.counters.cpu().numpy()[dr.C_CROSSINGS])
            what = f"direct pass of {args.sample_sources // 4} seeded star cells"
            del fs
        else:
            t0 = time.perf_counter()
            ref_run = oracle.run(m, pol, n_threads=nthreads)
            t_cpu = time.perf_counter() - t0
            got = f.U.cpu().numpy().astype(np.float64)
            ref_U = ref_run.U
            ref_cross = sum(int(r.counters[oracle.C_CROSS]) for r in ref_run.passes)
            gpu_cross = crossings
            what = f"full {wl.name} run (all passes)"
        nz = (np.abs(ref_U) > 0) | (np.abs(got) > 0)
        e = np.abs(got - ref_U)[nz] / np.maximum(np.abs(ref_U[nz]), 1e-300)
        parity = {"checked": what, "U_max_rel": float(e.max()), "U_p999_rel": float(np.quantile(e, 0.999)),
                  "crossings_gpu": gpu_cross, "crossings_oracle": ref_cross, "gate": 1e-4,
                  "pass": bool(e.max() <= 1e-4)}
        cpu = {"value": ref_cross * grid.n_lambda / t_cpu, "unit": "crossings*lambda/s", "cores": nthreads,
               "kind": "oracle", "sample": f"{what}, {ref_cross} crossings x {grid.n_lambda} wavelengths in {t_cpu:.1f} s"}
        log(f"oracle: {what} in {t_cpu:.1f} s; parity {parity}")

    # ---- timed steps
    def step():
        f.U.zero_()
        dr.run(G, pol, fields=f, collect=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    kinds = dr.PROF_STEP1 if pol.adaptive else dr.PROF_FIXED
    G.profile(kinds)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms, launches = G.profile_read()
    G.profile(0)

    ms_per_step = 1e3 * dt / args.steps
    value = cross_lambda / (dt / args.steps)
    # algorithmic bytes of the dominant march kernel per crossing: the
    # 64-byte leaf record read, and the energy-density row read-modify-write
    # (adaptive: n_lambda FP64 accumulators; fixed: one FP32 direction bin
    # per wavelength)
    if pol.adaptive:
        kern_cross = per_pass[0]
        per_cross = 64 + 2 * 8 * grid.n_lambda
        kernel = "k_march_adaptive (step 1)"
    else:
        kern_cross = crossings
        per_cross = 64 + 2 * 4 * grid.n_lambda
        kernel = f"k_march_fixed<{grid.n_lambda}>" if grid.n_lambda in (1, 4, 8, 16, 32, 64) else "k_march_fixed"
    launches_per_step = launches / args.steps
    avg_ms = kern_ms / max(launches, 1)
    achieved = (kern_cross * per_cross / launches_per_step) / (avg_ms * 1e-3) / 1e9
    # 64-byte atomic requests per crossing: one row of n_lambda FP64 (adaptive)
    # or FP32 (fixed) values.  A row narrower than 64 bytes shares its segment
    # with the rows of neighbouring cells, so its request count depends on which
    # lanes hit one segment, and no measured ceiling has that access pattern:
    # no atomic roofline is given then
    row_bytes = (8 if pol.adaptive else 4) * grid.n_lambda
    atomic_peak = ATOMIC_PEAK_ROWS_F64 if pol.adaptive else ATOMIC_PEAK_ROWS_F32
    if row_bytes >= 64:
        rpc = row_bytes / 64.0
        req_rate = rpc * (kern_cross / launches_per_step) / (avg_ms * 1e-3)
        atomic_roof = {"achieved": req_rate, "peak": atomic_peak, "unit": "64-byte atomic rows/s",
                       "frac": req_rate / atomic_peak, "requests_per_crossing": rpc}
    else:
        atomic_roof = {"achieved": None, "peak": None, "unit": "64-byte atomic rows/s", "frac": None,
                       "requests_per_crossing": None,
                       "note": f"{row_bytes}-byte rows share 64-byte segments; no matching ceiling"}
    traffic = None
    if wl.name == PMC_TRAFFIC["workload"] and sources_sha256() == PMC_TRAFFIC["sources_sha256"]:
        traffic = PMC_TRAFFIC["bytes_per_launch"]
    res = {
        "metric": "ray-cell crossings x lambda per second (1 MI355X) at rel err <= 1e-4 vs the FP64 oracle",
        "value": value,
        "unit": "crossings*lambda/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "description": wl.description, "cells": int(grid.n),
                   "n_lambda": int(grid.n_lambda),
                   "rays": (f"adaptive nside {pol.nside}..{pol.nside_max}, N_rays {pol.n_rays_min}, f_U {pol.f_U}"
                            if pol.adaptive else f"fixed nside {pol.nside}"),
                   "passes": (["step1"] if pol.adaptive and pol.step1 else []) + ["direct"] +
                             [f"scatter{k + 1}" for k in range(pol.n_scatter)],
                   "crossings_per_step": crossings, "crossings_per_pass": per_pass,
                   "balance_max_rel": balance, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel,
                     "avg_launch_ms": avg_ms, "bytes_per_crossing": per_cross,
                     "crossings_per_launch": kern_cross / launches_per_step},
        # the deposits are one 64-byte atomic request per crossing at 8 FP64
        # or 16 FP32 wavelengths (rocprofv3 TCC_ATOMIC equals the step-1
        # crossing count): the request rate against the measured ceiling is
        # the binding roofline of the march
        "atomic_roofline": atomic_roof,
        "cpu_baseline": cpu,
        "parity": parity,
    }
    if not args.no_extras:
        log("batched wavelengths ...")
        res["batched_lambda"] = batched_lambda(dr, W)
        log(f"batched wavelengths: {res['batched_lambda']}")
        log("batched models ...")
        res["batched_models"] = batched_models(dr, W)
        log(f"batched models: {res['batched_models']}")
        log("autotuner ...")
        res["autotune"] = autotuned(dr, W)
        log(f"autotuner: {res['autotune']}")
        log("adjoint ...")
        res["adjoint"] = adjoint_timing(dr, W)
        log(f"adjoint: {res['adjoint']}")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

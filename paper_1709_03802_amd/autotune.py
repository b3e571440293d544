"""Autotuner of the fixed-ray launch parameters (``dartray_tuning``).

The search is coordinate descent over a small discrete space: starting from
the defaults, each parameter in turn takes every candidate value with the
others held, the fastest is kept, and the sweep repeats until a sweep changes
nothing (at most ``rounds`` sweeps).  A candidate is timed with HIP events on
the grid's stream over whole passes (march, flush and bookkeeping), the
median of ``repeats`` timings.  Results are cached in a JSON file keyed by
device, cell count, wavelength count, ray Nside and pass kind.

The tuning changes speed only; every setting computes the same deposits up to
the order of FP32 additions (the library's tests check this).
"""

from __future__ import annotations

import json
import os
import statistics
from typing import Callable, Dict, List, Optional

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "dartray_tuning.json")

# parameter -> candidate values (0 = library default)
SPACE: Dict[str, List[int]] = {
    "lambda_tile": [0, 1, 4, 8, 16, 32],
    "block_waves": [4, 2, 1],
    "grid_blocks": [2048, 1024, 4096, 8192],
    "item_order": [0, 1],
    "dir_batch": [0, 192, 48],
}


def space_for(n_lambda: int) -> Dict[str, List[int]]:
    """Candidates that differ for this wavelength count (a tile at or above
    n_lambda is the same as all wavelengths)."""
    sp = {k: list(v) for k, v in SPACE.items()}
    sp["lambda_tile"] = [0] + [t for t in SPACE["lambda_tile"][1:] if t < n_lambda]
    return sp


def coordinate_search(space: Dict[str, List[int]], evaluate: Callable[[Dict[str, int]], float],
                      start: Optional[Dict[str, int]] = None, rounds: int = 2):
    """Minimise ``evaluate`` over the product of ``space`` by coordinate descent.

    Returns (best setting, best cost, list of (setting, cost) evaluated)."""
    cur = {k: v[0] for k, v in space.items()} if start is None else dict(start)
    seen: Dict[tuple, float] = {}
    log = []

    def cost(s):
        key = tuple(sorted(s.items()))
        if key not in seen:
            seen[key] = float(evaluate(dict(s)))
            log.append((dict(s), seen[key]))
        return seen[key]

    best = cost(cur)
    for _ in range(rounds):
        changed = False
        for k, vals in space.items():
            for v in vals:
                if v == cur[k]:
                    continue
                trial = dict(cur)
                trial[k] = v
                c = cost(trial)
                if c < best:
                    best, cur, changed = c, trial, True
        if not changed:
            break
    return cur, best, log


def cache_key(device: str, n: int, n_lambda: int, nside: int, kind: str) -> str:
    return f"{device}|n={n}|nl={n_lambda}|nside={nside}|{kind}"


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def save_cache(entries: dict, path: str = DEFAULT_CACHE) -> None:
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(entries, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_passes(G, policy, fields, repeats: int = 3, scatter: bool = True) -> float:
    """Median milliseconds of one pass (a scattering iteration, or the direct
    pass), timed with events on the grid's stream."""
    import torch
    from . import dartray as dr
    opts = dr.make_opts(policy, dr.MODE_DIRECT, counters=False)
    if scatter:
        dr.trace_direct(G, opts, fields)
    times = []
    for _ in range(repeats + 1):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(G.stream)
        if scatter:
            dr.scatter_iter(G, opts, fields, want_rk=False)
        else:
            dr.trace_direct(G, opts, fields)
        b.record(G.stream)
        b.synchronize()
        times.append(a.elapsed_time(b))
    return statistics.median(times[1:])


def tune(G, policy, cache_path: Optional[str] = DEFAULT_CACHE, rounds: int = 2, repeats: int = 3,
         scatter: bool = True, force: bool = False, verbose: bool = False):
    """Tune G's fixed-ray launch parameters for ``policy`` and apply them.

    Returns (setting, ms per pass, evaluations: list of (setting, ms)); an
    entry found in the cache is applied without timing (evaluations empty)."""
    import torch
    from . import dartray as dr
    if policy.adaptive:
        raise ValueError("the tuning covers fixed-ray passes")
    key = cache_key(torch.cuda.get_device_name(), G.n, G.nl, policy.nside, "scatter" if scatter else "direct")
    entries = load_cache(cache_path) if cache_path else {}
    if key in entries and not force:
        setting = entries[key]["setting"]
        G.set_tuning(**setting)
        return setting, entries[key]["ms"], []
    fields = dr.Fields(G)
    torch.cuda.synchronize()

    def evaluate(s):
        G.set_tuning(**s)
        ms = time_passes(G, policy, fields, repeats=repeats, scatter=scatter)
        if verbose:
            print(f"[autotune] {s}: {ms:.3f} ms", flush=True)
        return ms

    start = G.tuning().as_dict()
    start = {k: start[k] for k in SPACE}
    setting, ms, log = coordinate_search(space_for(G.nl), evaluate, start=start, rounds=rounds)
    G.set_tuning(**setting)
    if cache_path:
        entries = load_cache(cache_path)
        entries[key] = {"setting": setting, "ms": ms, "evaluations": len(log)}
        save_cache(entries, cache_path)
    return setting, ms, log

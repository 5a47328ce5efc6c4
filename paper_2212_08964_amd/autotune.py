"""Autotuner for grouped launches: picks the DP/Stream-K split by measurement.

The paper sizes the Stream-K grid with an analytical model and argues against
large per-shape kernel ensembles; for a grouped launch whose problem mix is
fixed (and replayed many times under a graph) a short measurement is cheap, so
this tuner times a small set of candidate schedules of the *same* kernel and
keeps the fastest:

* the automatic policy (model-chosen grid),
* pure data-parallel,
* basic Stream-K over every tile at grid p and at the model's grid,
* two-tile SK + DP and DP + one-tile SK,
* the hybrids with hybrid_min_waves = 1 (two-tile from one full wave on),

each with the planner's tile choice and with every compiled tile pinned, so
the tuner picks the tile shape and the DP/SK split together.

Each candidate is timed with HIP events over `reps` back-to-back launches
after a warm-up (best of three batches).  Decisions are cached in memory and,
if `cache_path` is given, in a JSON file keyed by device, dtypes, layouts and
the problem shapes.
"""
from __future__ import annotations

import hashlib
import json
import os

from . import skgemm as sk

_POLICIES = [
    dict(policy="auto"),
    dict(policy="dp"),
    dict(policy="sk"),
    dict(policy="2tile_sk_dp"),
    dict(policy="dp_1tile_sk"),
    dict(policy="2tile_sk_dp", hybrid_min_waves=1),
    dict(policy="auto", hybrid_min_waves=1),
]
# every policy with the planner's own tile choice, then with each compiled
# 16-bit tile configuration pinned (candidates a dtype does not compile are
# skipped)
TILES = [None, (256, 256, 64), (128, 128, 64, 4), (128, 128, 64, 8)]
CANDIDATES = [dict(c, tile=t) for t in TILES for c in _POLICIES]

_memo = {}


def _key(As, Bs, Cs):
    import torch
    dev = torch.cuda.get_device_name(As[0].device)
    shapes = tuple((A.shape[0], B.shape[1], A.shape[1]) for A, B in zip(As, Bs))
    lay = (sk._layout_of(As[0])[0], sk._layout_of(Bs[0])[0], sk._layout_of(Cs[0])[0])
    raw = json.dumps([dev, str(As[0].dtype), str(Cs[0].dtype), lay, shapes])
    return hashlib.sha1(raw.encode()).hexdigest()


def _time(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(3):
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / reps)
    return best * 1e3   # microseconds


def tune_grouped(As, Bs, Cs, reps=10, cache_path=None, candidates=None, verbose=False):
    """Returns (best options dict, {candidate label: microseconds})."""
    key = _key(As, Bs, Cs)
    if key in _memo:
        return _memo[key], {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            disk = json.load(fh)
        if key in disk:
            best = dict(disk[key])
            if best.get("tile"):
                best["tile"] = tuple(best["tile"])    # JSON keeps it as a list
            _memo[key] = best
            return best, {}
    results = {}
    best, best_t = None, float("inf")
    for cand in candidates or CANDIDATES:
        opts = dict(policy="auto", force_g=0, hybrid_min_waves=2, tile=None)
        opts.update(cand)
        label = json.dumps(opts, sort_keys=True)
        try:
            _, table = sk.grouped_matmul(As, Bs, Cs, **opts)
            t = _time(lambda: sk.grouped_matmul(As, Bs, Cs, table=table, **opts), reps)
        except sk.SkgemmError:
            continue
        results[label] = t
        if verbose:
            print(f"autotune {label}: {t:.1f} us", flush=True)
        if t < best_t:
            best, best_t = opts, t
    _memo[key] = best
    if cache_path:
        disk = {}
        if os.path.exists(cache_path):
            with open(cache_path) as fh:
                disk = json.load(fh)
        disk[key] = best
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as fh:
            json.dump(disk, fh, indent=1)
    return best, results

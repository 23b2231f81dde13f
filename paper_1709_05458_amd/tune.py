"""Tile autotuner: times candidate tile shapes of equal thread count on a
representative instance and keeps the fastest per (velocity set, precision,
walls, size class), cached in a JSON file (DUGKS_TUNE_CACHE, default
~/.cache/dugks/tune.json)."""
from __future__ import annotations

import json
import math
import os

from . import dugks

CANDIDATES_256 = [(32, 8), (16, 16), (64, 4), (8, 32)]


def _cache_path():
    return os.environ.get("DUGKS_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "dugks", "tune.json"))


def _load():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(d):
    p = _cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        with open(p + ".tmp", "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(p + ".tmp", p)
    except OSError:
        pass


def key_of(case, precision) -> str:
    walls = "periodic" if case.bc[0] == 0 and case.bc[2] == 0 else "walls"
    size = 2 ** int(round(math.log2(max(case.grid.nx, case.grid.ny))))
    return f"{case.vs.name}|p{precision}|{walls}|n{size}|{'u' if case.grid.is_uniform() else 'nu'}"


def time_tile(case, precision, tile, steps=6):
    import torch
    s = dugks.Solver(case, precision, tile=tile,
                     allow_defect=abs(case.vs.moment_defect()["sum_w_minus_1"]) > 1e-10)
    s.init_equilibrium(case.rho, case.ux, case.uy)
    s.step(2)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    s.step(steps)
    e1.record()
    torch.cuda.synchronize()
    s.close()
    return e0.elapsed_time(e1) / steps


def best_tile(case, precision, candidates=CANDIDATES_256, use_cache=True):
    """Fastest tile among `candidates` for this kind of instance (cached)."""
    cache = _load() if use_cache else {}
    k = key_of(case, precision)
    if k in cache:
        return tuple(cache[k]["tile"])
    times = {}
    for t in candidates:
        try:
            times[t] = time_tile(case, precision, t)
        except dugks.DugksError:
            continue
    best = min(times, key=times.get)
    cache[k] = {"tile": list(best), "ms_per_step": {f"{a}x{b}": v for (a, b), v in times.items()}}
    if use_cache:
        _save(cache)
    return best


def tiles_for(cases, precision):
    """Tuned 256-thread tiles for the lattice instances of a batch; None (the
    library's choice: one ring-tile shape for all of them, the one that
    launches the fewest threads) for the any-size instances."""
    out = []
    for c in cases:
        if c.vs.name in ("D2Q9", "D2Q37"):
            out.append(best_tile(c, precision))
        else:
            out.append(None)
    return out

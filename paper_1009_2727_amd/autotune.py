"""Tile shape and sort cadence of a run, chosen by timing short runs on the device.

Runs are grouped into classes by particles per cell and boost factor, the two inputs that set
how far particles drift across tiles between sorts and how much work a tile holds.  For each
class the tuner times a few steps of a trial run (the class's first workload, its grid capped
to keep the trial short, plasma pre-loaded) for every candidate tile shape at a fixed sort
cadence, then every candidate cadence at the best tile, and keeps the fastest pair.  The LDS
tile of the particle kernel holds a segment's box plus a 5-cell halo within 33 x 31 cells, so
the candidate tiles stay well inside it.
"""
from __future__ import annotations

import copy
import math

TILES = ((16, 8), (16, 16), (24, 8), (26, 8), (26, 12), (24, 16))
SORT_EVERY = (10, 20, 40, 80)


def run_class(workload) -> tuple:
    c, p = workload["config"], workload["plasma"]
    return (min(int(p["ppc"]) // 4, 3), int(round(math.log2(max(c["gamma_boost"], 1.0)))))


def time_steps(workload, tile, sort_every, steps=20, warmup=6) -> float:
    """Device milliseconds per step of `workload` with the given tile and sort cadence."""
    import torch
    from . import Sim
    sim = Sim.from_workload(workload, tile=tile, sort_every=sort_every)
    sim.step(warmup)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(sim.stream)
    sim.step(steps)
    b.record(sim.stream)
    torch.cuda.synchronize()
    if sim.sync_status() != 0:
        return math.inf
    return a.elapsed_time(b) / steps


def trial_workload(workload, max_nx=160, max_nz=1024):
    w = copy.deepcopy(workload)
    c = w["config"]
    c["nx"] = min(c["nx"], max_nx)
    c["nz"] = min(c["nz"], max_nz)
    w["plasma"]["start_um"] = -1e30          # pre-loaded: the steady state of the window
    w["plasma"]["ramp_um"] = 0.0
    return w


class Autotuner:
    def __init__(self, tiles=TILES, sort_every=SORT_EVERY, steps=20, warmup=6):
        self.tiles, self.sorts, self.steps, self.warmup = tiles, sort_every, steps, warmup
        self.cache: dict = {}
        self.trials: dict = {}

    def tune(self, workload) -> dict:
        key = run_class(workload)
        if key in self.cache:
            return self.cache[key]
        w = trial_workload(workload)
        base = 20 if 20 in self.sorts else self.sorts[0]
        tile_ms = {t: time_steps(w, t, base, self.steps, self.warmup) for t in self.tiles}
        tile = min(tile_ms, key=tile_ms.get)
        sort_ms = {k: (tile_ms[tile] if k == base else time_steps(w, tile, k, self.steps, self.warmup))
                   for k in self.sorts}
        sort_every = min(sort_ms, key=sort_ms.get)
        best = {"tile": tile, "sort_every": sort_every, "ms_per_step": sort_ms[sort_every],
                "class": key}
        self.trials[key] = {"tiles": {f"{a}x{b}": v for (a, b), v in tile_ms.items()},
                            "sort_every": sort_ms}
        self.cache[key] = best
        return best

    def tune_all(self, workloads) -> list:
        return [self.tune(w) for w in workloads]

"""Autotuner of the fused-pass schedule (the SQNGD_SCHED_* hint of a batch).

Every schedule computes the same results; they differ in how the (row,
Doppler bin, partner) work of the fused pass is cut into wavefronts and
blocks, which changes the number of gradient partials too. The tuner times
whole outer iterations (HIP-graph replays on the current stream, HIP events)
of the batch under each candidate and returns the fastest; results are cached
per device and batch shape, in memory and optionally in a JSON file.
"""
from __future__ import annotations

import json
import os

import torch

from . import native as nat

CANDIDATES = (nat.SCHED_THROUGHPUT, nat.SCHED_SPLIT8, nat.SCHED_SPLIT12, nat.SCHED_SPLIT16)
_cache: dict = {}


def signature(probs) -> str:
    shapes = sorted((p["M"], p["N"], p["L"], p["F"]) for p in probs)
    return f"{torch.cuda.get_device_name()}|{len(probs)}|" + ";".join(f"{m},{n},{l},{f}" for m, n, l, f in shapes)


def _time_steps(probs, opt, seeds, steps: int, per_graph: int = 10) -> float:
    from . import optim
    run = optim.SQNGD(probs, opt, seeds=seeds)
    run.capture(per_graph)
    run.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(1, steps // per_graph)
    e0.record()
    for _ in range(reps):
        run.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / (reps * per_graph)


def tune(probs, opt, steps: int = 40, cache_path: str | None = None) -> tuple:
    """(best schedule, {schedule: ms per outer iteration}) for this batch."""
    key = signature(probs)
    disk = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            disk = json.load(f)
    if key in _cache:
        return _cache[key]
    if key in disk:
        _cache[key] = (int(disk[key]["best"]), {int(k): v for k, v in disk[key]["ms"].items()})
        return _cache[key]
    seeds = list(range(len(probs)))
    times = {}
    for c in CANDIDATES:
        times[c] = _time_steps([dict(p, schedule=c) for p in probs], opt, seeds, steps)
    best = min(times, key=times.get)
    _cache[key] = (best, times)
    if cache_path:
        disk[key] = {"best": best, "ms": {str(k): v for k, v in times.items()}}
        with open(cache_path, "w") as f:
            json.dump(disk, f, indent=1)
    return best, times

"""Autotuner of the fused-pass schedule, per FFT-length group of a batch.

Every schedule computes the same results; they differ in how the (row,
Doppler bin, partner) work of the fused pass is cut into wavefronts and
blocks (SQNGD_SCHED_* hints, include/sqngd.h). The choices are per group of
problems with the same FFT length: at 512 the throughput pass or the latency
variant with 4, 8, 12 or 16 waves per block, at 1024 the throughput pass or
the latency variant with 2, 4 or 8, elsewhere the throughput pass; and for the batch, the
throughput groups in one launch or one launch per group. The tuner times
whole outer iterations (HIP-graph replays on the current stream, HIP events)
in a coordinate search -- every group's candidates with the others fixed,
then the launch grouping -- and returns one hint per problem. Results are
cached per device architecture and batch shape, in memory and in a JSON file.
"""
from __future__ import annotations

import json
import os

import torch

from . import native as nat

SPLIT_SHAPES = {512: (nat.SCHED_SPLIT4, nat.SCHED_SPLIT8, nat.SCHED_SPLIT12, nat.SCHED_SPLIT16),
                1024: (nat.SCHED_SPLIT2, nat.SCHED_SPLIT4, nat.SCHED_SPLIT8)}
# the pair form (one block per (row, Doppler bin, partner)) at the FFT lengths
# whose transform spans a block, while each problem's F M partial rows fit
PAIR_LENGTHS = (2048, 4096)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_2604_25728_amd", "tune.json")
_cache: dict = {}


def fft_len(N: int) -> int:
    P = 128
    while P < 2 * N - 1:
        P *= 2
    return P


def arch() -> str:
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", "") or p.name


def signature(probs) -> str:
    shapes = sorted((p["M"], p["N"], p["L"], p["F"]) for p in probs)
    return f"{arch()}|{len(probs)}|" + ";".join(f"{m},{n},{l},{f}" for m, n, l, f in shapes)


def candidates(probs) -> dict:
    """{FFT length: candidate hints} of the batch's groups."""
    out = {}
    for P in sorted({fft_len(p["N"]) for p in probs}):
        mmax = max(p["M"] for p in probs if fft_len(p["N"]) == P)
        out[P] = [nat.SCHED_THROUGHPUT] + [c for c in SPLIT_SHAPES.get(P, ()) if mmax <= c]
        if P in PAIR_LENGTHS and all(p["F"] * p["M"] <= 4096 for p in probs if fft_len(p["N"]) == P):
            out[P].append(nat.SCHED_PAIR)
    return out


def hints_for(probs, choice: dict, fused: bool) -> list:
    """One hint per problem: its group's choice, with FUSED (the throughput
    groups in one launch) or GROUPED (one launch per group) in place of
    THROUGHPUT."""
    out = []
    for p in probs:
        h = choice[fft_len(p["N"])]
        if h == nat.SCHED_THROUGHPUT:
            h = nat.SCHED_FUSED if fused else nat.SCHED_GROUPED
        out.append(h)
    return out


def _time_steps(probs, opt, seeds, steps: int, per_graph: int) -> float:
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


def tune(probs, opt, steps: int = 20, per_graph: int = 10, cache_path: str | None = DEFAULT_CACHE) -> tuple:
    """(one hint per problem, {description: ms per outer iteration}) for this batch."""
    key = signature(probs)
    if key in _cache:
        return _cache[key]
    disk = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                disk = json.load(f)
        except (OSError, ValueError):
            disk = {}
    if key in disk:
        _cache[key] = (list(disk[key]["hints"]), dict(disk[key]["ms"]))
        return _cache[key]
    seeds = list(range(len(probs)))
    cands = candidates(probs)
    choice = {P: c[0] for P, c in cands.items()}
    fused = False
    times = {}

    def run(ch, fu):
        name = ",".join(f"{P}:{ch[P]}" for P in sorted(ch)) + ("|fused" if fu else "")
        if name not in times:
            ps = [dict(p, schedule=h) for p, h in zip(probs, hints_for(probs, ch, fu))]
            times[name] = _time_steps(ps, opt, seeds, steps, per_graph)
        return times[name]

    best = run(choice, fused)
    for P, cs in cands.items():
        for c in cs[1:]:
            trial = dict(choice)
            trial[P] = c
            t = run(trial, fused)
            if t < best:
                best, choice = t, trial
    if sum(1 for P in cands if P <= 2048 and choice[P] == nat.SCHED_THROUGHPUT) >= 2:
        t = run(choice, True)
        if t < best:
            best, fused = t, True
    hints = hints_for(probs, choice, fused)
    _cache[key] = (hints, times)
    if cache_path:
        disk[key] = {"hints": hints, "ms": times}
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            with open(cache_path, "w") as f:
                json.dump(disk, f, indent=1)
        except OSError:
            pass
    return hints, times

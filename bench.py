#!/usr/bin/env python
"""Throughput of the SQNGD hot path on one MI355X.

A step is one outer iteration of Algorithm 1 over one batch (sqngd_step: for
every design one filter update and one logit update, each a full AF loss +
gradient evaluation -- quantisation, fused FFT AF / loss / adjoint pass,
reduction, optimiser), recorded once in a HIP graph and replayed. The default
workload is the uneven batch: 64 independent designs with N drawn from
{128, 256, 512, 1024}, M from {2, 4, 8}, L from {4, 8, 16}, F = 129 Doppler
bins over [-0.5, 0.5], every delay in the region of interest, p = 16, each
with 8 random restarts (512 problems). Inputs are seeded synthetic N(0,1)
logits and the matched filter, resident in HBM before the timed region.

The metric's evaluation is one loss + one gradient evaluation of one problem
(a step holds two per problem: the filter step's grad_h and the logit step's
grad_z). The line also carries the rate of evaluations with both gradients
(sqngd_af_backward with grad_z and grad_h) on the same batch.

Prints one JSON line with the metric, the roofline of the dominant kernel and
the oracle timed on the host cores. Diagnostics go to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X published FP32 vector peak
HBM_PEAK_GBPS = 8000.0            # MI355X published HBM3E bandwidth
COPY_BYTES = 1 << 28              # calibration copy of the counter runs: 256 MiB read, 256 MiB written
# HBM traffic of the dominant fused-pass kernel from the committed counter
# summaries (two rocprofv3 --pmc passes each), per workload
TRAFFIC_FILES = {"uneven": os.path.join(ROOT, "profiles", "k_pass_2048_uneven_64x8_traffic.md"),
                 "m4n256": os.path.join(ROOT, "profiles", "k_pass_split_m4n256_traffic.md"),
                 "wide_m8n1024": os.path.join(ROOT, "profiles", "k_pass_2048_wide_m8n1024_traffic.md")}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def fft_len(N: int) -> int:
    P = 128
    while P < 2 * N - 1:
        P *= 2
    return P


def pass_flops(prob: dict) -> float:
    """Algorithmic FP32 flops of one fused pass with gradient for one problem:
    per unit (self row, Doppler bin) 2M+2 length-P FFTs at 5 P log2 P flops
    each, plus about 30 flops per delay cell and partner for the products,
    the magnitude, the p-norm terms and the adjoint accumulation."""
    M, F, P = prob["M"], prob["F"], fft_len(prob["N"])
    units = M * F
    return units * ((2 * M + 2) * 5.0 * P * math.log2(P) + M * 30.0 * P)


def cube_cells(prob: dict) -> int:
    return prob["M"] ** 2 * prob["F"] * (2 * prob["N"] - 1)


# Cube-equivalent bytes of one evaluation: what a pipeline that materialises
# the AF cube would move per cell (complex64 A written and read back for the
# loss, complex64 adjoint G written and read back for the gradient).
CUBE_BYTES_PER_CELL = 32


def cube_frac(cells: int, evals_per_cell_set: float, ms: float) -> float:
    """Cube-equivalent bandwidth of `evals_per_cell_set` evaluations of
    `cells` cells in `ms` milliseconds, as a fraction of the HBM peak."""
    return CUBE_BYTES_PER_CELL * cells * evals_per_cell_set / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS


def time_graph(run, steps: int, warmup: int, per_graph: int):
    """ms per outer iteration over `steps` iterations run as graph replays of
    `per_graph` iterations each (steps is rounded up to a multiple): (mean,
    wall seconds, iterations, per-replay ms per iteration). Every replay is
    bracketed by HIP events on the stream it runs on."""
    import numpy as np
    import torch
    run.capture(per_graph)
    for _ in range(max(1, warmup // per_graph)):
        run.replay()
    torch.cuda.synchronize()
    reps = max(1, -(-steps // per_graph))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(reps):
        run.replay()
        ev[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([ev[i].elapsed_time(ev[i + 1]) / per_graph for i in range(reps)])
    return ev[0].elapsed_time(ev[-1]) / (reps * per_graph), wall, reps * per_graph, per


def spread(per) -> dict:
    import numpy as np
    return {"median": float(np.median(per)), "p10": float(np.percentile(per, 10)),
            "p90": float(np.percentile(per, 90)), "replays": int(len(per))}


def launch_durations(run, nat, steps: int, repeat: int = 1) -> dict:
    """Mean duration (ms) of the batch's fused-pass launches over `steps`
    eager steps (two passes each), keyed by the FFT lengths each launch
    covers (one launch may cover several groups): HIP events recorded by the
    library on the launch stream around `repeat` back-to-back launches of that
    pass (identical inputs and outputs), divided by `repeat`."""
    import numpy as np
    import torch
    n = 2 * steps * 6
    torch.cuda.synchronize()
    nat.profile_enable(n, repeat)
    for _ in range(steps):
        run.step()
    torch.cuda.synchronize()
    d = nat.profile_read(n)
    masks = nat.profile_groups(n)
    nat.profile_enable(0, 1)
    out = {}
    for m in sorted(set(masks.tolist())):
        Ps = tuple(128 << g for g in range(6) if (m >> g) & 1)
        out[Ps] = float(np.mean(d[masks == m]))
    return out


def source_hash() -> str:
    """sha256 over the device sources and their launch code (kernels, FFT,
    plan layout, launcher): a stored traffic figure is used only while the
    kernels and launch shapes it was measured on are unchanged."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2604_25728_amd", "csrc")
    for name in ("api.hip", "fft_wave.hpp", "kernels.hip", "plan.hpp"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def stored_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary of
    `workload`, or None when the summary is missing, names another kernel or
    was taken on other sources."""
    try:
        with open(TRAFFIC_FILES[workload]) as f:
            txt = f.read()
    except (OSError, KeyError):
        return None
    vals = {}
    for line in txt.splitlines():
        if line.startswith(("traffic_bytes_per_launch:", "source_hash:", "kernel:")):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_hash") != source_hash() or "traffic_bytes_per_launch" not in vals:
        return None
    if vals.get("kernel") != kernel:
        return None
    return float(vals["traffic_bytes_per_launch"])


def counter_run(run, steps: int):
    """Workload for the rocprofv3 --pmc passes: `steps` eager iterations (every
    kernel a separate dispatch), then a plain device copy of COPY_BYTES that
    calibrates FETCH_SIZE / WRITE_SIZE."""
    import torch
    for _ in range(steps):
        run.step()
    torch.cuda.synchronize()
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"counter run: {steps} eager iterations, then one copy of {COPY_BYTES} bytes")


def cpu_model() -> dict:
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}


def _oracle_step_seconds(prob: dict, opt: dict, seed: int) -> float:
    import numpy as np

    from oracle import sqngd_ref as R
    from paper_2604_25728_amd import inputs as I
    R.build()
    z = I.logits(prob["M"], prob["N"], prob["L"], seed).astype(np.float64)
    h = R.matched_init(z)
    state = R.new_state(prob["M"], prob["N"], prob["L"])
    t0 = time.perf_counter()
    R.step(prob, opt, z, h, state, 0)
    return time.perf_counter() - t0


def oracle_cost(prob: dict) -> float:
    """Work of one oracle outer iteration in the direct sums' unit: two
    evaluations of M^2 F N^2 delay-Doppler products each."""
    return 2.0 * prob["M"] ** 2 * prob["F"] * prob["N"] ** 2


def cpu_baseline(designs, opt: dict, budget_s: float) -> dict:
    """The FP64 oracle's outer iteration (two evaluations, each the AF cube,
    the loss and both gradients by direct sums) timed on the host cores on a
    bounded sample of the batch: its distinct shapes in increasing cost until
    the budget is spent. The direct sums cost M^2 F N^2 products per
    evaluation, so the per-product time of the sample (least squares through
    the origin) prices the whole batch; the rate is scaled to the metric's
    evaluations (two per problem per outer iteration)."""
    import numpy as np
    shapes = {}
    for p, sd in designs:
        shapes.setdefault((p["M"], p["N"], p["L"]), (p, sd))
    order = sorted(shapes.values(), key=lambda ps: oracle_cost(ps[0]))
    xs, ts, names = [], [], []
    t0 = time.perf_counter()
    for p, sd in order:
        if ts and time.perf_counter() - t0 + ts[-1] * oracle_cost(p) / xs[-1] > budget_s:
            break
        ts.append(_oracle_step_seconds(p, opt, sd))
        xs.append(oracle_cost(p))
        names.append(f"M={p['M']} N={p['N']} L={p['L']}")
    el = time.perf_counter() - t0
    xs, ts = np.array(xs), np.array(ts)
    per = float((xs * ts).sum() / (xs * xs).sum())
    batch_s = per * sum(oracle_cost(p) for p, _ in designs)
    cores = int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)))
    return {"value": 2 * len(designs) / batch_s, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": f"one oracle outer iteration of each of the {len(xs)} cheapest distinct shapes of the "
                      f"batch ({', '.join(names)}; {el:.1f} s), {per * 1e9:.3f} ns per delay-Doppler product "
                      f"(M^2 F N^2 per evaluation), priced over the {len(designs)} problems: "
                      f"{batch_s:.0f} s per outer iteration of the batch",
            "s_per_batch_iteration": batch_s, "ns_per_product": per * 1e9,
            "sample_shapes": names, "sample_seconds": ts.tolist(), **cpu_model()}


def cpu_single_thread(designs, opt: dict, budget_s: float) -> dict:
    """The same leg in a child process restricted to one OpenMP thread."""
    code = ("import json, sys; sys.path.insert(0, %r); import bench; from paper_2604_25728_amd import inputs as I; "
            "d = I.uneven_designs(); print(json.dumps(bench.cpu_baseline(d, I.config('m4n256')['opt'], %r)))"
            % (ROOT, budget_s))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                         timeout=30 * budget_s + 120)
    if out.returncode != 0:
        return {"error": out.stderr[-400:]}
    r = json.loads(out.stdout.strip().splitlines()[-1])
    return {k: r[k] for k in ("value", "unit", "cores", "sample", "ns_per_product")}


def fft_route_eval(s, h, prob: dict, workers: int = 1) -> tuple:
    """One evaluation by the paper's FFT route (eq. 33-36) in complex128 with
    scipy's pocketfft, vectorised over (m, l, f): loss, and the packed
    gradients with respect to the waveforms and the filters (the adjoint of
    every linear step: the delay selection, the inverse FFT, the product with
    the conjugate filter spectra, the zero-padded forward FFTs and the Doppler
    modulation), plus the SNRL term. A CPU baseline of the GPU path's own
    algorithm, not a reference: its values are checked against the oracle."""
    import numpy as np
    import scipy.fft as sf
    s, h = np.asarray(s, np.complex128), np.asarray(h, np.complex128)
    M, N = s.shape
    F, P = prob["F"], fft_len(N)
    nu = prob["nu_min"] + np.arange(F) * ((prob["nu_max"] - prob["nu_min"]) / (F - 1) if F > 1 else 0.0)
    n = np.arange(N)
    mod = np.exp(2j * np.pi * np.outer(nu, n) / N)                       # [F][N]
    X = sf.fft(s[:, None, :] * mod[None], n=P, axis=-1, workers=workers)  # [M][F][P]
    H = sf.fft(h, n=P, axis=-1, workers=workers)                          # [M][P]
    r = sf.ifft(X[:, None] * np.conj(H)[None, :, None], axis=-1, workers=workers)  # [M][M][F][P]
    tau = np.arange(-(N - 1), N)
    k = (-tau) % P
    A = r[..., k]                                                         # [M][M][F][2N-1]
    mask = (tau >= prob["tau_lo"]) & (tau <= prob["tau_hi"])
    mask = np.broadcast_to(mask, A.shape).copy()
    for m in range(M):
        mask[m, m, :, N - 1] = False
    a = np.abs(A) / N * mask
    amax = a.max()
    p = prob["p"]
    lp = amax * ((a / amax) ** p).sum() ** (1.0 / p)
    c = (np.conj(h) * s).sum(axis=1)
    p_tar = 10 ** (-prob["snrl_target_db"] / 20)
    pm = np.abs(c) / N
    loss = prob["w_psl"] * lp + prob["w_snrl"] * ((pm - p_tar) ** 2).mean()
    with np.errstate(divide="ignore", invalid="ignore"):
        G = np.where(mask, prob["w_psl"] * lp ** (1 - p) * a ** (p - 2) * A / N ** 2, 0.0)
    gr = np.zeros(r.shape, np.complex128)
    gr[..., k] = G                                                        # adjoint of the selection
    gy = sf.fft(gr, axis=-1, workers=workers) / P                         # adjoint of the inverse FFT
    gX = (H[None, :, None] * gy).sum(axis=1)                              # [M][F][P]
    gs = (np.conj(mod)[None] * (P * sf.ifft(gX, axis=-1, workers=workers)[..., :N])).sum(axis=1)
    gH = (X[:, None] * np.conj(gy)).sum(axis=(0, 2))                      # [M][P]
    gh = P * sf.ifft(gH, axis=-1, workers=workers)[..., :N]
    gS = prob["w_snrl"] * (2.0 / M) * (pm - p_tar) * c / (N * np.abs(c))
    gs = gs + gS[:, None] * h
    gh = gh + np.conj(gS)[:, None] * s
    return loss, gs, gh


def cpu_fft_route(prob: dict, budget_s: float) -> dict:
    """The FFT route of fft_route_eval timed on the host cores (scipy workers)."""
    import numpy as np
    from paper_2604_25728_amd import inputs as I
    cores = len(os.sched_getaffinity(0))
    s = np.exp(2j * np.pi * np.random.default_rng(0).random((prob["M"], prob["N"])))
    h = I.complex_gaussian(prob["M"], prob["N"], 1).astype(np.complex128)
    n = 0
    t0 = time.perf_counter()
    while n < 1 or time.perf_counter() - t0 < budget_s:
        fft_route_eval(s, h, prob, workers=cores)
        n += 1
    el = time.perf_counter() - t0
    return {"value": n / el, "unit": "evals/s", "cores": cores, "kind": "fft_route_numpy",
            "sample": f"{n} evaluations (loss, both gradients) by the FFT route in complex128, {el:.1f} s"}


def transmit_extras(I, torch, only=None) -> dict:
    """The paper's transmit side at its Table VI shape (M=2 N=512 B=4 F=129,
    r_n = 100, c = 300, N_h = N_x = 10, |tau| <= 50): one design, SQNAF, and 64
    stacked restarts, each one outer iteration per HIP graph replay."""
    extras = {}
    from paper_2604_25728_amd import sqnnative as SN
    for key, matched, R in (("paper_sqn_m2n512_b4", False, 1), ("paper_sqnaf_m2n512_b4", True, 1),
                            ("paper_sqn_m2n512_b4_x64", False, 64)):
        if only is not None and key != only:
            continue
        # SQNAF: the AF extension of SQN (matched filters, no step A), at 0 dB SNRL
        ps = I.make_problem(2, 512, 4, 129, p=16.0, w_psl=0.1, w_snrl=0.9,
                            **({"snrl_target_db": 0.0} if matched else {}))
        os_ = I.make_opt(lr_z=1e-5, lr_h=5e-2, n_h=10, n_x=10, total_iters=2000)
        d = SN.SQNDesign(ps, os_, copies=100, c=300.0, seed=list(range(R)), matched=matched)
        d.batch.set_roi_weights([I.roi_window_weights(ps, 50)] * R)
        d.capture()              # one outer iteration as a HIP graph
        d.graph.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            d.graph.replay()
        e1.record()
        torch.cuda.synchronize()
        ms_it = e0.elapsed_time(e1) / 5
        evals = (10 if matched else 20) * R
        extras[key] = {
            "ms_per_outer_iteration": ms_it, "evals_per_s": evals / (ms_it * 1e-3),
            "projected_s_for_2000_iterations": 2000 * ms_it * 1e-3,
            "designs": R,
            "shape": {"M": 2, "N": 512, "B": 4, "F": 129, "copies": 100, "c": 300.0,
                      "n_h": 0 if matched else 10, "n_x": 10, "matched_filter": matched}}
        log(f"paper {'SQNAF' if matched else 'SQN'} M=2 N=512 B=4 x{R}: {ms_it:.2f} ms per outer iteration")
        del d
    return extras


def roofline_of(probs, ldur: dict, workload: str, hints=None) -> dict:
    """Roofline record of the batch's dominant fused-pass launch (the launch
    with the largest measured duration): the algorithmic flops of that launch
    (pass_flops summed over the problems of the FFT lengths it covers) over
    its measured mean duration, against the FP32 vector peak."""
    Ps = max(ldur, key=ldur.get)
    sel = [p for p in probs if fft_len(p["N"]) in Ps]
    flops = sum(pass_flops(p) for p in sel)
    ms = ldur[Ps]
    achieved = flops / (ms * 1e-3) / 1e12
    kernel = "k_pass_multi<3, false>" if len(Ps) > 1 else f"k_pass<{Ps[0]}, 3, false>"
    traffic = stored_traffic(workload, kernel)
    return {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic,
            "kernel": f"{kernel} (fused AF + loss + adjoint over FFT lengths {list(Ps)})",
            "kernel_us": ms * 1e3, "flops_per_launch": flops, "problems_in_launch": len(sel),
            "traffic_source": os.path.relpath(TRAFFIC_FILES[workload], ROOT) if traffic else None,
            "launch_us": {"+".join(str(P) for P in k): v * 1e3 for k, v in sorted(ldur.items())}}


def both_gradient_rate(probs, seeds, reps: int = 5) -> dict:
    """Evaluations with both gradients (sqngd_af_backward: loss, grad_z of the
    soft waveform and grad_h) of every problem of the batch, timed with HIP
    events around `reps` back-to-back calls."""
    import torch

    from paper_2604_25728_amd import inputs as I
    from paper_2604_25728_amd import native as nat
    b = nat.Batch(probs)
    z = b.pack_z([I.logits(p["M"], p["N"], p["L"], s) for p, s in zip(probs, seeds)])
    _, x = b.hard_quantize(z, want_idx=False)
    stats = b.new_stats()
    b.af_backward(z, x, nat.WAVE_SOFT, stats=stats)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.af_backward(z, x, nat.WAVE_SOFT, stats=stats)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"evals_per_s": len(probs) / (ms * 1e-3), "ms_per_batch": ms,
            "unit": "evaluations with the loss, grad_z and grad_h of one problem per second"}


def single_design(I, nat, optim, name: str, steps: int, tuned: bool) -> dict:
    """One design of a preset: ms per outer iteration (graph replays of ten
    iterations each, as the optimiser runs between stopping checks), its
    fused pass's roofline."""
    c = I.config(name)
    prob, opt = c["problem"], c["opt"]
    sched = None
    if tuned:
        from paper_2604_25728_amd import tune
        hints, sched_ms = tune.tune([prob], opt, steps=40)
        sched = hints[0]
        log(f"{name}: schedule tuning (ms per step): " +
            ", ".join(f"{k}: {v * 1e3:.1f} us" for k, v in sched_ms.items()) + f" -> {sched}")
    run = optim.SQNGD([prob], opt, seeds=[0], schedule=sched)
    ms, _, n, per = time_graph(run, steps, 20, 10)
    import numpy as np
    import torch
    torch.cuda.synchronize()
    nat.profile_enable(2 * 50, 20)
    for _ in range(50):
        run.step()
    torch.cuda.synchronize()
    kd = float(np.mean(nat.profile_read(100)))
    nat.profile_enable(0, 1)
    flops = pass_flops(prob)
    achieved = flops / (kd * 1e-3) / 1e12
    kname = (f"k_pass_split<{fft_len(prob['N'])}, 3, {int(sched)}, false>" if sched and sched >= 8
             else f"k_pass<{fft_len(prob['N'])}, 3, false>")
    traffic = stored_traffic(name, kname)
    out = {"ms_per_step": ms, **{f"step_{k}": v for k, v in spread(per).items()},
           "evals_per_s": 2.0 / (ms * 1e-3),
           "cube_equiv_frac_of_hbm": cube_frac(cube_cells(prob), 2, ms),
           "shape": {k: prob[k] for k in ("M", "N", "L", "F", "nu_min", "nu_max")},
           "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                        "kernel": kname, "kernel_us": kd * 1e3, "flops_per_launch": flops},
           "pass_cube_equiv_frac_of_hbm": CUBE_BYTES_PER_CELL * cube_cells(prob) / (kd * 1e-3) / 1e9 / HBM_PEAK_GBPS}
    if sched is not None:
        out["schedule"] = int(sched)
    log(f"{name}: step {ms * 1e3:.1f} us, pass {kd * 1e3:.2f} us = {achieved:.2f} TFLOP/s")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the other workloads and the copy probe")
    ap.add_argument("--transmit", nargs="?", const="all", default=None,
                    choices=["all", "paper_sqn_m2n512_b4", "paper_sqnaf_m2n512_b4", "paper_sqn_m2n512_b4_x64"],
                    help="time only the transmit-side workloads (all, or one) and print them as one JSON line")
    ap.add_argument("--counters", action="store_true",
                    help="run the workload for rocprofv3 --pmc (eager iterations + calibration copy) and exit")
    ap.add_argument("--workload", default="uneven",
                    choices=["uneven", "m4n256", "wide_m8n1024", "paper_m2n512_roi50", "paper_m2n1200_roi50"],
                    help="workload of a --counters run (paper_m2n512_roi50 / paper_m2n1200_roi50: one design at "
                         "M=2 N=512 L=4 / N=1200 L=16, F=129, with the |tau| <= 50 window as ROI weights)")
    ap.add_argument("--schedule", type=int, default=12,
                    help="fused-pass schedule hint of an m4n256 --counters run (the timed run tunes it)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the designs of a batch "
              "are independent, and a multi-GPU run would shard them without communication",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2604_25728_amd import inputs as I
    from paper_2604_25728_amd import native as nat
    from paper_2604_25728_amd import optim

    torch.cuda.set_device(0)
    log(f"device: {torch.cuda.get_device_name(0)}")
    designs = I.uneven_designs()
    probs = [p for p, _ in designs]
    seeds = [sd for _, sd in designs]
    opt = I.config("m4n256")["opt"]

    if args.transmit:
        only = None if args.transmit == "all" else args.transmit
        print(json.dumps({"transmit_side": transmit_extras(I, torch, only)}), flush=True)
        return
    if args.counters:
        if args.workload == "uneven":
            run = optim.SQNGD(probs, opt, seeds=seeds)
        elif args.workload in ("paper_m2n512_roi50", "paper_m2n1200_roi50"):
            pp = (I.make_problem(2, 512, 4, 129, p=16.0) if args.workload == "paper_m2n512_roi50"
                  else I.make_problem(2, 1200, 16, 129, p=16.0))
            run = optim.SQNGD([pp], opt, seeds=[0], roi_weights=[I.roi_window_weights(pp, 50)])
        else:
            c = I.config(args.workload)
            sched = args.schedule if args.workload == "m4n256" else None
            run = optim.SQNGD([c["problem"]], c["opt"], seeds=[0], schedule=sched)
        counter_run(run, args.steps)
        return

    # ---- the headline: one outer iteration of the uneven 512-problem batch per step,
    # with the fused-pass schedule of each FFT-length group tuned on the device
    from paper_2604_25728_amd import tune
    hints, tune_ms = tune.tune(probs, opt)
    log("schedule tuning (ms per step): " + ", ".join(f"{k}: {v:.2f}" for k, v in tune_ms.items()))
    run = optim.SQNGD(probs, opt, seeds=seeds, schedule=hints)
    ms_step, wall, steps, per = time_graph(run, args.steps, args.warmup, 1)
    evals = 2 * len(probs)
    log(f"uneven x{len(probs)}: step {ms_step:.3f} ms ({steps} graph replays of one iteration, wall {wall:.3f} s)")
    ldur = launch_durations(run, nat, 2)
    roof = roofline_of(probs, ldur, "uneven")
    log(f"dominant pass {roof['kernel']}: {roof['kernel_us']:.1f} us, {roof['achieved']:.2f} TFLOP/s; launches "
        + ", ".join(f"{k}: {v:.0f} us" for k, v in roof["launch_us"].items()))
    del run
    both = both_gradient_rate([dict(p, schedule=h) for p, h in zip(probs, hints)], seeds)
    log(f"both gradients: {both['ms_per_batch']:.2f} ms per batch evaluation")
    cells = sum(cube_cells(p) for p in probs)

    extras = {}
    if not args.no_extras:
        extras["m4n256_x1"] = single_design(I, nat, optim, "m4n256", 500, True)
        extras["wide_m8n1024_x1"] = single_design(I, nat, optim, "wide_m8n1024", 50, False)
        prob = I.config("m4n256")["problem"]
        R = 64
        runb = optim.SQNGD([prob] * R, opt, seeds=list(range(R)))
        msb, _, _, _ = time_graph(runb, 20, 5, 1)
        extras["m4n256_x64"] = {"designs": R, "ms_per_step": msb, "evals_per_s": 2.0 * R / (msb * 1e-3),
                                "cube_equiv_frac_of_hbm": cube_frac(R * cube_cells(prob), 2, msb)}
        log(f"m4n256 x{R}: step {msb * 1e3:.1f} us")
        del runb
        c = I.config("m4n512")
        r = optim.SQNGD([c["problem"]] * 64, c["opt"], seeds=list(range(64)))
        ms_c, _, _, _ = time_graph(r, 20, 5, 1)
        extras["m4n512_x64"] = {"ms_per_step": ms_c, "evals_per_s": 2.0 * 64 / (ms_c * 1e-3),
                                "cube_equiv_frac_of_hbm": cube_frac(64 * cube_cells(c["problem"]), 2, ms_c)}
        log(f"m4n512 x64: step {ms_c * 1e3:.1f} us")
        del r
        # the paper's own shapes: N = 1200 (FFT length 4096), M = 2, B = 16 phase
        # levels, 129 Doppler bins in [-0.5, 0.5], the fixed ROI |tau| <= 50 as 0/1
        # weights w(tau, f) (eq. 8-9), one design and 64 restarts; and Table III's
        # widest span, nu in [-600, 600] on the 1201-bin integer grid
        pp = I.make_problem(2, 1200, 16, 129, p=16.0)
        ww = I.roi_window_weights(pp, 50)
        for count in (1, 64):
            r = optim.SQNGD([pp] * count, opt, seeds=list(range(count)), roi_weights=[ww] * count)
            ms_c, _, _, _ = time_graph(r, 20 if count == 1 else 10, 5, 1)
            extras[f"paper_m2n1200_roi50_x{count}"] = {
                "ms_per_step": ms_c, "evals_per_s": 2.0 * count / (ms_c * 1e-3),
                "cube_equiv_frac_of_hbm": cube_frac(count * cube_cells(pp), 2, ms_c),
                "shape": {"M": 2, "N": 1200, "L": 16, "F": 129, "roi": "|tau| <= 50 as weights"}}
            log(f"M=2 N=1200 |tau|<=50 x{count}: step {ms_c * 1e3:.1f} us")
            del r
        pw = I.make_problem(2, 1200, 16, 1201, nu_min=-600.0, nu_max=600.0, p=16.0)
        r = optim.SQNGD([pw], opt, seeds=[0], roi_weights=[I.roi_window_weights(pw, 50)])
        ms_c, _, _, _ = time_graph(r, 10, 3, 1)
        extras["paper_m2n1200_wide600_roi50_x1"] = {
            "ms_per_step": ms_c, "evals_per_s": 2.0 / (ms_c * 1e-3),
            "cube_equiv_frac_of_hbm": cube_frac(cube_cells(pw), 2, ms_c),
            "shape": {"M": 2, "N": 1200, "L": 16, "F": 1201, "nu": [-600, 600], "roi": "|tau| <= 50 as weights"}}
        log(f"M=2 N=1200 nu in [-600, 600] F=1201: step {ms_c:.3f} ms")
        del r
        # the paper's own transmit side (ResNet + copied staircase, Sec. III-A) at
        # its Table VI shape and settings
        extras.update(transmit_extras(I, torch))
        n = 1 << 28
        a = torch.empty(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        extras["hbm_copy_GBps"] = 10 * 2 * 4 * n / (e0.elapsed_time(e1) * 1e-3) / 1e9
        del a, b

    out = {
        "metric": "AF loss+grad evals/s",
        "value": evals / (ms_step * 1e-3),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "step_ms": spread(per),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "uneven batch: 64 designs x 8 random restarts (512 problems), N in {128, 256, "
                               "512, 1024}, M in {2, 4, 8}, L in {4, 8, 16}, F=129 nu in [-0.5, 0.5], all delays, "
                               "p=16; one outer iteration (filter step + logit step) per step, one HIP graph replay "
                               "per step; fused-pass schedule per FFT-length group from the autotuner",
                   "designs": 64, "restarts": 8, "problems": len(probs), "evals_per_step": evals,
                   "schedule": {str(fft_len(p["N"])): h for p, h in zip(probs, hints)},
                   "eval_unit": "one loss + one gradient evaluation of one problem (grad_h in the filter step, "
                                "grad_z in the logit step)"},
        "roofline": roof,
        "both_gradients": both,
        "cube_equivalent": {"bytes_per_eval_batch": CUBE_BYTES_PER_CELL * cells,
                            "step_GBps": 2 * CUBE_BYTES_PER_CELL * cells / (ms_step * 1e-3) / 1e9,
                            "step_frac_of_hbm": cube_frac(cells, 2, ms_step)},
    }
    if extras:
        out["extras"] = extras
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(designs, opt, args.cpu_seconds)
        log(f"cpu baseline: {out['cpu_baseline']['value']:.4f} evals/s on {out['cpu_baseline']['cores']} cores")
        out["cpu_baseline"]["single_thread"] = cpu_single_thread(designs, opt, 0.25 * args.cpu_seconds)
        prob = I.config("m4n256")["problem"]
        out["cpu_fft_route_m4n256"] = cpu_fft_route(prob, min(5.0, args.cpu_seconds))
        log(f"cpu FFT route (M=4 N=256): {out['cpu_fft_route_m4n256']['value']:.1f} evals/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

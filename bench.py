#!/usr/bin/env python
"""Throughput of the SQNGD hot path on one MI355X.

A step is one outer iteration of Algorithm 1 (sqngd_step with one filter
update and one logit update, each a full AF loss + gradient evaluation:
quantisation, fused FFT AF / loss / adjoint pass, reduction, optimiser),
recorded once in a HIP graph and replayed. The default workload is one design
of M=4 waveforms, N=256 chips, L=8 phase levels, F=129 Doppler bins over
[-0.5, 0.5], every delay in the region of interest, p=16, temperature annealed
1.0 -> 0.05. Inputs are seeded synthetic N(0,1) logits and the matched filter;
they are resident in HBM before the timed region starts.

Prints one JSON line with the metric, the roofline of the fused pass kernel
and the oracle timed on the host cores.
Diagnostics go to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X published FP32 vector peak
HBM_PEAK_GBPS = 8000.0            # MI355X published HBM3E bandwidth
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pass_split_m4n256_traffic.md")
COPY_BYTES = 1 << 28              # calibration copy of the counter runs: 256 MiB read, 256 MiB written


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
    `per_graph` iterations each (steps is rounded up to a multiple)."""
    import torch
    run.capture(per_graph)
    for _ in range(max(1, warmup // per_graph)):
        run.replay()
    torch.cuda.synchronize()
    reps = max(1, -(-steps // per_graph))
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(reps):
        run.replay()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / (reps * per_graph), wall, reps * per_graph


def kernel_durations(run, nat, steps: int, repeat: int = 20):
    """Per-launch durations (ms) of the fused pass over `steps` eager steps: HIP
    events on the launch stream around `repeat` back-to-back launches of each
    pass (identical inputs and outputs), divided by `repeat`."""
    import torch
    torch.cuda.synchronize()
    nat.profile_enable(2 * steps, repeat)
    for _ in range(steps):
        run.step()
    torch.cuda.synchronize()
    d = nat.profile_read(2 * steps)
    nat.profile_enable(0, 1)
    return d


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


def stored_traffic(schedule: int):
    """HBM bytes per fused-pass launch from the committed counter summary, or
    None when the summary is missing or was taken on other sources or under
    another schedule."""
    try:
        with open(TRAFFIC_FILE) as f:
            txt = f.read()
    except OSError:
        return None
    vals = {}
    for line in txt.splitlines():
        if line.startswith(("traffic_bytes_per_launch:", "source_hash:", "schedule:")):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_hash") != source_hash() or "traffic_bytes_per_launch" not in vals:
        return None
    if int(vals.get("schedule", "-1")) != int(schedule):
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


def cpu_baseline(prob: dict, opt: dict, budget_s: float) -> dict:
    """The FP64 oracle's outer iteration, timed on the host cores."""
    import numpy as np

    from oracle import sqngd_ref as R
    from paper_2604_25728_amd import inputs as I
    R.build()
    z = I.logits(prob["M"], prob["N"], prob["L"], 0).astype(np.float64)
    h = R.matched_init(z)
    state = R.new_state(prob["M"], prob["N"], prob["L"])
    n = 0
    t0 = time.perf_counter()
    while n < 1 or time.perf_counter() - t0 < budget_s:
        z, h, state, _, _ = R.step(prob, opt, z, h, state, n)
        n += 1
    el = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)))
    return {"value": 2 * n / el, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} outer iterations (2 evaluations each: AF cube, loss and both gradients "
                      f"by FP64 direct sums) of the same workload, {el:.1f} s"}


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


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--iters-per-graph", type=int, default=10,
                    help="outer iterations recorded in one HIP graph (one sqngd_run call)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched and copy probes")
    ap.add_argument("--schedule", type=int, default=12,
                    help="fused-pass schedule hint of the --counters run (the timed run tunes it)")
    ap.add_argument("--transmit", nargs="?", const="all", default=None,
                    choices=["all", "paper_sqn_m2n512_b4", "paper_sqnaf_m2n512_b4", "paper_sqn_m2n512_b4_x64"],
                    help="time only the transmit-side workloads (all, or one) and print them as one JSON line")
    ap.add_argument("--counters", action="store_true",
                    help="run the workload for rocprofv3 --pmc (eager iterations + calibration copy) and exit")
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
    cfg = I.config("m4n256")
    prob, opt = cfg["problem"], cfg["opt"]
    log(f"device: {torch.cuda.get_device_name(0)}")

    if args.transmit:
        only = None if args.transmit == "all" else args.transmit
        print(json.dumps({"transmit_side": transmit_extras(I, torch, only)}), flush=True)
        return
    if args.counters:
        run = optim.SQNGD([prob], opt, seeds=[0], schedule=args.schedule)
        counter_run(run, args.steps)
        return
    from paper_2604_25728_amd import tune
    sched, sched_ms = tune.tune([prob], opt, steps=40)
    log("schedule tuning (ms per step): " + ", ".join(f"{k}: {v * 1e3:.1f} us" for k, v in sched_ms.items())
        + f" -> {sched}")
    run = optim.SQNGD([prob], opt, seeds=[0], schedule=sched)
    ms_step, wall, steps = time_graph(run, args.steps, args.warmup, args.iters_per_graph)
    evals_per_s = 2.0 / (ms_step * 1e-3)
    log(f"step {ms_step * 1e3:.2f} us ({steps} iterations in graphs of {args.iters_per_graph}, "
        f"wall {wall:.3f} s)")

    kd = kernel_durations(run, nat, min(args.steps, 200))
    kd_avg_ms = float(kd.mean())
    traffic = stored_traffic(sched)
    flops = pass_flops(prob)
    achieved = flops / (kd_avg_ms * 1e-3) / 1e12
    log(f"fused pass: {kd.size} launches, mean {kd_avg_ms * 1e3:.2f} us, "
        f"{achieved:.2f} TFLOP/s algorithmic")
    cube_gbps = CUBE_BYTES_PER_CELL * cube_cells(prob) / (kd_avg_ms * 1e-3) / 1e9
    cube_step_gbps = 2 * CUBE_BYTES_PER_CELL * cube_cells(prob) / (ms_step * 1e-3) / 1e9

    extras = {}
    if not args.no_extras:
        R = 64
        runb = optim.SQNGD([prob] * R, opt, seeds=list(range(R)))
        msb, _, _ = time_graph(runb, max(10, args.steps // 10), 5, args.iters_per_graph)
        kdb = kernel_durations(runb, nat, 20)
        extras["batched_restarts"] = {
            "designs": R, "ms_per_step": msb, "evals_per_s": 2.0 * R / (msb * 1e-3),
            "cube_equiv_frac_of_hbm": cube_frac(R * cube_cells(prob), 2, msb),
            "pass_kernel_us": float(kdb.mean() * 1e3),
            "pass_tflops": R * flops / (kdb.mean() * 1e-3) / 1e12}
        log(f"batched x{R}: step {msb * 1e3:.1f} us, {extras['batched_restarts']['evals_per_s']:.0f} evals/s")
        del runb
        # the other workloads: one wide-span design, the network's design size
        # batched, and the uneven 64-design x 8-restart batch
        for name, count in (("wide_m8n1024", 1), ("m4n512", 64)):
            c = I.config(name)
            r = optim.SQNGD([c["problem"]] * count, c["opt"], seeds=list(range(count)))
            ms_c, _, _ = time_graph(r, 20, 10, 10)
            extras[f"{name}_x{count}"] = {"ms_per_step": ms_c, "evals_per_s": 2.0 * count / (ms_c * 1e-3),
                                          "cube_equiv_frac_of_hbm": cube_frac(count * cube_cells(c["problem"]),
                                                                              2, ms_c),
                                          "shape": {k: c["problem"][k] for k in ("M", "N", "L", "F")}}
            log(f"{name} x{count}: step {ms_c * 1e3:.1f} us")
            del r
        designs = I.uneven_designs()
        r = optim.SQNGD([p for p, _ in designs], I.config("m4n256")["opt"], seeds=[sd for _, sd in designs])
        ms_c, _, _ = time_graph(r, 10, 10, 10)
        extras["uneven_64x8"] = {"ms_per_step": ms_c, "evals_per_s": 2.0 * len(designs) / (ms_c * 1e-3),
                                   "cube_equiv_frac_of_hbm": cube_frac(sum(cube_cells(p) for p, _ in designs),
                                                                       2, ms_c),
                                   "designs": 64, "restarts": 8}
        log(f"uneven x{len(designs)}: step {ms_c * 1e3:.1f} us")
        del r
        # the paper's own shapes: N = 1200 (FFT length 4096), M = 2, B = 16 phase
        # levels, 129 Doppler bins in [-0.5, 0.5], the fixed ROI |tau| <= 50 as 0/1
        # weights w(tau, f) (eq. 8-9), one design and 64 restarts
        pp = I.make_problem(2, 1200, 16, 129, p=16.0)
        ww = I.roi_window_weights(pp, 50)
        for count in (1, 64):
            r = optim.SQNGD([pp] * count, opt, seeds=list(range(count)), roi_weights=[ww] * count)
            ms_c, _, _ = time_graph(r, 20 if count == 1 else 10, 10, 10)
            extras[f"paper_m2n1200_roi50_x{count}"] = {
                "ms_per_step": ms_c, "evals_per_s": 2.0 * count / (ms_c * 1e-3),
                "cube_equiv_frac_of_hbm": cube_frac(count * cube_cells(pp), 2, ms_c),
                "shape": {"M": 2, "N": 1200, "L": 16, "F": 129, "roi": "|tau| <= 50 as weights"}}
            log(f"M=2 N=1200 |tau|<=50 x{count}: step {ms_c * 1e3:.1f} us")
            del r
        # the paper's own transmit side (ResNet + copied staircase, Sec. III-A) at
        # its Table VI shape and settings: M=2 N=512 B=4, r_n=100, c=300,
        # N_h = N_x = 10, eps = 0.1 (w_psl 0.1, w_snrl 0.9), SNRL target 0.5 dB,
        # |tau| <= 50 as ROI weights, 129 Doppler bins in [-0.5, 0.5]
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
        "value": evals_per_s,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "one SQNGD design, M=4 N=256 L=8 F=129 nu in [-0.5,0.5], all 511 "
                               "delays, p=16, one filter + one logit update per step, HIP graphs of "
                               f"{args.iters_per_graph} steps",
                   "M": prob["M"], "N": prob["N"], "L": prob["L"], "F": prob["F"],
                   "p": prob["p"], "evals_per_step": 2, "schedule": int(sched)},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
                     "traffic": traffic, "kernel": "k_pass_split (fused AF + loss + adjoint)",
                     "kernel_us": kd_avg_ms * 1e3, "flops_per_launch": flops,
                     "traffic_source": os.path.relpath(TRAFFIC_FILE, ROOT) if traffic else None},
        "cube_equivalent": {"GBps": cube_gbps, "frac_of_hbm": cube_gbps / HBM_PEAK_GBPS,
                            "bytes_per_eval": CUBE_BYTES_PER_CELL * cube_cells(prob),
                            "step_GBps": cube_step_gbps, "step_frac_of_hbm": cube_step_gbps / HBM_PEAK_GBPS},
    }
    if extras:
        out["extras"] = extras
    if not args.no_cpu_baseline:
        out["cpu_fft_route"] = cpu_fft_route(prob, min(10.0, args.cpu_seconds))
        log(f"cpu FFT route: {out['cpu_fft_route']['value']:.1f} evals/s on {out['cpu_fft_route']['cores']} cores")
        out["cpu_baseline"] = cpu_baseline(prob, opt, args.cpu_seconds)
        log(f"cpu baseline: {out['cpu_baseline']['value']:.3f} evals/s on {out['cpu_baseline']['cores']} cores")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

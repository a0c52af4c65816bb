"""Learned warm start for the SQNGD optimiser (not part of the paper's method).

The paper starts every design from random phases and reparameterises it with
a ResNet trained for that design alone (Sec. III-A, eq. 17; Algorithm 1,
initialisation). Here a small 1-D conv network (netnative.Net, BF16 MFMA
kernels) is trained once, on converged runs of the optimiser, to propose the
starting logits of new designs; plain N(0,1) logits stay the fallback, and the
plain optimiser's PSL judges the proposal.

Pairing. A deterministic network regressed from independent noise onto
unrelated solutions would learn their mean. So each training run i starts from
logits that are a fixed function of its own noise eps_i[M][N]:
    z0[m][n][l] = cos(2 pi (l / L - Phi(eps_i[m][n]))),  Phi the normal CDF,
and its target is the hard phase indices the optimiser reaches from there: a
function of eps_i, learned with a per-chip cross-entropy.

Time to target (per held-out seed s): the random arm starts from N(0,1)
logits of seed s and runs the full iteration budget; its final hard PSL is the
target. The warm arm feeds the noise of seed s through the network and runs
from the proposed logits. For both arms the first checkpoint (every
`check_every` iterations) at which the hard PSL is at or below the target with
the worst SNRL at or below 0.5 dB is the time to target. Seconds are timed per
design: a subset of the seeds runs one design at a time in each arm, each
checkpoint's iterations, its hard evaluation and (warm arm) the network's
proposal bracketed by HIP events.

Workload: M=4 N=512 L=8 F=129 with the paper's weighting eps = 0.1 and the
SNRL target 0.3 dB, inside the 0.5 dB bound (inputs preset m4n512_ws).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch
from scipy.special import ndtr

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    __package__ = "paper_2604_25728_amd"

from . import inputs as I  # noqa: E402
from . import netnative as NN  # noqa: E402
from . import optim  # noqa: E402


def log(*a):
    print(*a, flush=True)


def paired_logits(eps: np.ndarray, L: int) -> np.ndarray:
    """z0[m][n][l] = cos(2 pi (l / L - Phi(eps[m][n]))) as float32."""
    u = ndtr(np.asarray(eps, dtype=np.float64))
    lv = np.arange(L, dtype=np.float64) / L
    return np.cos(2.0 * np.pi * (lv[None, None, :] - u[..., None])).astype(np.float32)


def cond_of(prob: dict):
    return (prob["L"] / 8.0, prob["nu_max"] - prob["nu_min"])


PARAMS_M4N512 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "warmstart_m4n512.npy")
WORKLOAD = "m4n512_ws"


def trained_params(path: str = PARAMS_M4N512) -> np.ndarray:
    """Parameters of the network trained on converged M=4 N=512 L=8 F=129 runs
    (written by `train-eval --save-params`), float32."""
    return np.load(path, allow_pickle=False)


def generate(prob: dict, opt: dict, seeds, batch: int, iters: int) -> dict:
    """Converged runs from the paired starts: hard indices and final stats."""
    M, N, L = prob["M"], prob["N"], prob["L"]
    idx, psl, snrl = [], [], []
    seeds = list(seeds)
    t0 = time.perf_counter()
    for c in range(0, len(seeds), batch):
        part = seeds[c: c + batch]
        z0 = [paired_logits(I.noise(M, N, s), L) for s in part]
        run = optim.SQNGD([prob] * len(part), opt, z0=z0)
        run.run(iters, use_graph=True, iters_per_graph=10)
        for a in run.hard_indices():
            idx.append(a.astype(np.uint8))
        for st in run.hard_stats():
            psl.append(st["pslr_db"])
            snrl.append(st["snrl_db_max"])
        torch.cuda.synchronize()
        log(f"generate: {c + len(part)}/{len(seeds)} runs, {time.perf_counter() - t0:.1f} s, "
            f"median PSL {np.median(psl):.2f} dB")
        del run
    return {"seeds": np.array(seeds, dtype=np.int64), "idx": np.stack(idx), "psl_db": np.array(psl),
            "snrl_db": np.array(snrl)}


def train(prob: dict, data: dict, epochs: int, batch: int, lr: float, seed: int = 0) -> tuple:
    """Network trained on (noise of seed, hard indices) pairs; returns it and the loss history."""
    M, N, L = prob["M"], prob["N"], prob["L"]
    net = NN.Net(M, N, L, batch, cond=cond_of(prob), seed=seed)
    seeds = data["seeds"]
    noise_all = torch.tensor(np.stack([I.noise(M, N, int(s)) for s in seeds]), device="cuda")
    tgt_all = torch.tensor(data["idx"].astype(np.int32), device="cuda")
    rng = np.random.default_rng(seed)
    hist = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = rng.permutation(len(seeds))
        losses = []
        for c in range(0, len(order) - batch + 1, batch):
            sel = torch.tensor(order[c: c + batch], device="cuda")
            net.train_step(noise_all.index_select(0, sel), tgt_all.index_select(0, sel), lr=lr)
            losses.append(net.loss.clone())
        ep_loss = float(torch.stack(losses).mean().item())
        hist.append(ep_loss)
        log(f"train: epoch {ep + 1}/{epochs} loss {ep_loss:.4f} ({time.perf_counter() - t0:.1f} s)")
    return net, hist


def propose(net_params: torch.Tensor, prob: dict, seeds) -> tuple:
    """Proposed starting logits for the seeds' noise (one network call) and its GPU time in ms."""
    M, N, L = prob["M"], prob["N"], prob["L"]
    net = NN.Net(M, N, L, len(seeds), cond=cond_of(prob), params=net_params)
    noise = torch.tensor(np.stack([I.noise(M, N, int(s)) for s in seeds]), device="cuda")
    net.forward(noise)  # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    z = net.forward(noise)
    e1.record()
    torch.cuda.synchronize()
    return [z[i].cpu().numpy() for i in range(len(seeds))], e0.elapsed_time(e1)


def trajectory(prob: dict, opt: dict, z0, iters: int, check_every: int) -> tuple:
    """Hard PSL / SNRL of every design at each checkpoint, and the GPU ms per iteration."""
    run = optim.SQNGD([prob] * len(z0), opt, z0=z0)
    psl, snrl = [], []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    gpu_ms = 0.0
    for it in range(0, iters, check_every):
        e0.record()
        run.run(check_every, use_graph=True, iters_per_graph=check_every if check_every <= 50 else 10)
        e1.record()
        st = run.hard_stats()
        torch.cuda.synchronize()
        gpu_ms += e0.elapsed_time(e1)
        psl.append([s["pslr_db"] for s in st])
        snrl.append([s["snrl_db_max"] for s in st])
    return np.array(psl).T, np.array(snrl).T, gpu_ms / iters


def first_hit(psl_row, snrl_row, target, snrl_bound, check_every):
    ok = np.nonzero((psl_row <= target + 1e-6) & (snrl_row <= snrl_bound + 1e-6))[0]
    return int((ok[0] + 1) * check_every) if ok.size else None


def seconds_to_target(prob: dict, opt: dict, z0, target: float, snrl_bound: float, iters: int, check_every: int,
                      extra_ms: float = 0.0):
    """One design alone: GPU seconds until its hard PSL is at or below `target`
    with the worst SNRL within the bound (checkpoints every `check_every`
    iterations: the iterations as one graph replay and the hard evaluation,
    bracketed by HIP events), plus `extra_ms`; None if not reached."""
    run = optim.SQNGD([prob], opt, z0=[z0])
    run.capture(check_every)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms = extra_ms
    for _ in range(0, iters, check_every):
        e0.record()
        run.replay()
        stats = run.batch.af_forward(run.z, run.h, 1)
        e1.record()
        torch.cuda.synchronize()
        ms += e0.elapsed_time(e1)
        st = optim.nat.decode_stats(stats.cpu().numpy())[0]
        if st["pslr_db"] <= target + 1e-6 and st["snrl_db_max"] <= snrl_bound + 1e-6:
            return ms / 1e3
    return None


def time_to_target(prob: dict, opt: dict, net_params: torch.Tensor, seeds, iters: int, check_every: int,
                   snrl_max_db: float = 0.5, timed_seeds: int = 0) -> dict:
    M, N, L = prob["M"], prob["N"], prob["L"]
    seeds = list(seeds)
    zr = [I.logits(M, N, L, int(s)) for s in seeds]
    psl_r, snrl_r, ms_r = trajectory(prob, opt, zr, iters, check_every)
    zw, net_ms = propose(net_params, prob, seeds)
    psl_w, snrl_w, ms_w = trajectory(prob, opt, zw, iters, check_every)
    per = []
    for i in range(len(seeds)):
        target = psl_r[i, -1]
        hr = first_hit(psl_r[i], snrl_r[i], target, snrl_max_db, check_every)
        hw = first_hit(psl_w[i], snrl_w[i], target, snrl_max_db, check_every)
        per.append({"seed": int(seeds[i]), "target_psl_db": float(target), "snrl_bound_db": float(snrl_max_db),
                    "random_iters": hr, "warm_iters": hw, "warm_start_psl_db": float(psl_w[i, 0]),
                    "random_start_psl_db": float(psl_r[i, 0]), "warm_final_psl_db": float(psl_w[i, -1]),
                    "random_final_snrl_db": float(snrl_r[i, -1]), "warm_final_snrl_db": float(snrl_w[i, -1])})
    # seeds whose random run ends within the SNRL bound define a target
    valid = [p for p in per if p["random_iters"] is not None]
    reached = [p for p in valid if p["warm_iters"] is not None]
    ratios = [p["warm_iters"] / p["random_iters"] for p in reached]
    per_design_ms = ms_w / len(seeds)
    res = {
        "seeds": len(seeds), "iters_budget": iters, "check_every": check_every, "snrl_bound_db": snrl_max_db,
        "random_within_bound": len(valid) / len(seeds),
        "fraction_reached": len(reached) / max(1, len(valid)),
        "median_ratio_iters": float(np.median(ratios)) if ratios else None,
        "median_random_iters": float(np.median([p["random_iters"] for p in valid])) if valid else None,
        "median_warm_iters": float(np.median([p["warm_iters"] for p in reached])) if reached else None,
        "median_target_psl_db": float(np.median(psl_r[:, -1])),
        "median_warm_final_psl_db": float(np.median(psl_w[:, -1])),
        "median_random_final_snrl_db": float(np.median(snrl_r[:, -1])),
        "median_warm_final_snrl_db": float(np.median(snrl_w[:, -1])),
        "gpu_ms_per_iteration_batch": ms_w, "gpu_ms_per_design_iteration": per_design_ms,
        "network_ms_batch": net_ms,
        "per_seed": per,
    }
    if timed_seeds:
        sec_r, sec_w, sub = [], [], [p for p in valid][:timed_seeds]
        for p in sub:
            i = seeds.index(p["seed"])
            sec_r.append(seconds_to_target(prob, opt, zr[i], p["target_psl_db"], snrl_max_db, iters, check_every))
            z1, one_ms = propose(net_params, prob, [p["seed"]])
            sec_w.append(seconds_to_target(prob, opt, z1[0], p["target_psl_db"], snrl_max_db, iters, check_every,
                                           extra_ms=one_ms))
        pairs = [(a, b) for a, b in zip(sec_r, sec_w) if a is not None and b is not None]
        res.update({"timed_seeds": len(sub),
                    "timed_median_random_seconds": float(np.median([a for a, _ in pairs])) if pairs else None,
                    "timed_median_warm_seconds": float(np.median([b for _, b in pairs])) if pairs else None,
                    "timed_median_ratio_seconds": float(np.median([b / a for a, b in pairs])) if pairs else None,
                    "timed_warm_reached": sum(b is not None for b in sec_w) / max(1, len(sub)),
                    "timed_per_seed": [{"seed": p["seed"], "random_s": a, "warm_s": b}
                                       for p, a, b in zip(sub, sec_r, sec_w)]})
    return res


def main():
    ap = argparse.ArgumentParser(description="warm-start data generation, training and time-to-target")
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate")
    g.add_argument("--runs", type=int, default=4096)
    g.add_argument("--first-seed", type=int, default=100000)
    g.add_argument("--iters", type=int, default=2000)
    g.add_argument("--batch", type=int, default=512)
    g.add_argument("--out", required=True)
    t = sub.add_parser("train-eval")
    t.add_argument("--data", required=True)
    t.add_argument("--epochs", type=int, default=30)
    t.add_argument("--batch", type=int, default=64)
    t.add_argument("--lr", type=float, default=2e-3)
    t.add_argument("--eval-seeds", type=int, default=256)
    t.add_argument("--iters", type=int, default=2000)
    t.add_argument("--check-every", type=int, default=50)
    t.add_argument("--out", required=True)
    t.add_argument("--save-params", default=None, help="write the trained parameters (.npy, float32)")
    t.add_argument("--timed-seeds", type=int, default=32, help="seeds timed one design at a time per arm")
    args = ap.parse_args()
    cfg = I.config(WORKLOAD)
    prob, opt = cfg["problem"], dict(cfg["opt"])
    if args.cmd == "generate":
        opt["total_iters"] = args.iters
        data = generate(prob, opt, range(args.first_seed, args.first_seed + args.runs), args.batch, args.iters)
        np.savez_compressed(args.out, **data)
        log(f"wrote {args.out}")
        return
    d = np.load(args.data)
    data = {k: d[k] for k in d.files}
    opt["total_iters"] = args.iters
    net, hist = train(prob, data, args.epochs, args.batch, args.lr)
    if args.save_params:
        np.save(args.save_params, net.params.cpu().numpy().astype(np.float32), allow_pickle=False)
    res = time_to_target(prob, opt, net.params, range(args.eval_seeds), args.iters, args.check_every,
                         timed_seeds=args.timed_seeds)
    res["train_loss"] = hist
    res["train_runs"] = int(len(data["seeds"]))
    res["train_median_psl_db"] = float(np.median(data["psl_db"]))
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
    summ = {k: v for k, v in res.items() if k != "per_seed"}
    log(json.dumps(summ))


if __name__ == "__main__":
    main()

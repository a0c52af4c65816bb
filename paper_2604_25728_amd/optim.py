"""Driver of the alternating SQNGD iteration (Algorithm 1) on one GPU.

Every outer iteration is one ``sqngd_step`` of the C ABI; the driver owns the
device tensors (logits, filters, Adam state, step counter, statistics),
optionally records one iteration in a HIP graph (``torch.cuda.CUDAGraph`` is
hipGraph on ROCm) and replays it, and saves or restores the complete state.
"""
from __future__ import annotations

import numpy as np
import torch

from . import inputs as I
from . import native as nat


class SQNGD:
    """A batch of independent designs optimised together.

    probs: list of problem dicts (inputs.make_problem); opt: option dict
    (inputs.make_opt); seeds: one seed per problem for the N(0,1) logits, or
    z0: a list of [M][N][L] float32 arrays to start from instead."""

    def __init__(self, probs, opt: dict, seeds=None, z0=None, device="cuda", schedule=None, roi_weights=None):
        """schedule: None keeps each problem's hint (default automatic), an
        int applies that SQNGD_SCHED_* hint to every problem, a list gives one
        hint per problem, "tune" times the candidates per FFT-length group
        first (tune.tune) and applies the fastest. roi_weights: one [F][2N-1]
        array (or None) per problem, the w(tau, f) of eq. 8-9."""
        if isinstance(schedule, str) and schedule == "tune":
            from . import tune
            schedule, _ = tune.tune(probs, opt)
        if isinstance(schedule, (list, tuple)):
            probs = [dict(p, schedule=int(h)) for p, h in zip(probs, schedule)]
        elif schedule is not None:
            probs = [dict(p, schedule=int(schedule)) for p in probs]
        self.schedule = schedule
        self.batch = nat.Batch(probs, device=device)
        if roi_weights is not None:
            self.batch.set_roi_weights(roi_weights)
        self.probs = self.batch.probs
        self.opt_dict = dict(opt)
        self.opt = nat.make_opt(opt)
        if z0 is None:
            seeds = list(range(len(probs))) if seeds is None else list(seeds)
            z0 = [I.logits(p["M"], p["N"], p["L"], s) for p, s in zip(self.probs, seeds)]
        self.z = self.batch.pack_z(z0)
        # filters start as the matched filter of the hard starting waveform
        # (Algorithm 1's initialisation); |x_m|^2 = N, so the projection of
        # eq. 32 leaves them unchanged.
        _, x = self.batch.hard_quantize(self.z, want_idx=False)
        self.h = x.clone()
        dev = self.batch.device
        self.adam = torch.zeros(self.batch.adam_floats, dtype=torch.float32, device=dev)
        self.counter = torch.zeros(1, dtype=torch.int32, device=dev)
        self.stats = self.batch.new_stats(2 * self.batch.n)
        self.graph = None
        self.graph_iters = 0

    # ------------------------------------------------------------------ steps
    def step(self, n_iters: int = 1):
        """Enqueue n_iters outer iterations (one sqngd_run call) on the current stream."""
        if n_iters == 1:
            self.batch.step(self.opt, self.z, self.h, self.adam, self.counter, self.stats)
        else:
            self.batch.run(self.opt, n_iters, self.z, self.h, self.adam, self.counter, self.stats)

    def capture(self, iters_per_graph: int = 1):
        """Record iters_per_graph outer iterations in a HIP graph; replay() runs them."""
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step(iters_per_graph)
        self.graph = g
        self.graph_iters = iters_per_graph
        return g

    def replay(self):
        self.graph.replay()

    def run(self, iters: int, use_graph: bool = True, iters_per_graph: int = 10):
        """iters outer iterations: graph replays of iters_per_graph iterations, then the rest eagerly."""
        if not use_graph:
            done = 0
            while done < iters:
                k = min(iters_per_graph, iters - done)
                self.step(k)
                done += k
            return
        if self.graph is None or self.graph_iters != iters_per_graph:
            self.capture(iters_per_graph)
        for _ in range(iters // iters_per_graph):
            self.graph.replay()
        if iters % iters_per_graph:
            self.step(iters % iters_per_graph)

    def subset(self, keep) -> "SQNGD":
        """A new driver over the problems `keep` (indices into this batch) that
        continues from their current state: logits, filters, Adam moments and
        the shared iteration counter t (so the temperature schedule goes on)."""
        keep = [int(i) for i in keep]
        new = SQNGD.__new__(SQNGD)
        new.schedule = self.schedule
        new.batch = nat.Batch([self.probs[i] for i in keep], device=self.batch.device)
        if self.batch.roi_w is not None:
            new.batch.set_roi_weights([self.batch.unpack_roi(i).cpu().numpy() for i in keep])
        new.probs = new.batch.probs
        new.opt_dict = dict(self.opt_dict)
        new.opt = nat.make_opt(self.opt_dict)
        new.z = torch.cat([self.batch.unpack_z(self.z, i).reshape(-1) for i in keep])
        new.h = torch.cat([self.batch.unpack_w(self.h, i).reshape(-1) for i in keep])
        new.adam = torch.cat([self.batch.unpack_adam(self.adam, i) for i in keep])
        new.counter = self.counter.clone()
        new.stats = new.batch.new_stats(2 * new.batch.n)
        new.graph = None
        new.graph_iters = 0
        return new

    # ------------------------------------------------------------- inspection
    @property
    def t(self) -> int:
        return int(self.counter.item())

    def step_stats(self):
        """(step A stats, step B stats) of the last iteration, per problem."""
        st = nat.decode_stats(self.stats.cpu().numpy())
        n = self.batch.n
        return st[:n], st[n:]

    def hard_stats(self):
        """Statistics of the hard-quantised designs with the current filters."""
        stats = self.batch.af_forward(self.z, self.h, nat.WAVE_HARD)
        return nat.decode_stats(stats.cpu().numpy())

    def hard_indices(self):
        idx, _ = self.batch.hard_quantize(self.z, want_x=False)
        return [self.batch.unpack_w(idx, i).cpu().numpy() for i in range(self.batch.n)]

    # ------------------------------------------------------------- checkpoint
    def state_dict(self) -> dict:
        return {"z": self.z.detach().cpu().clone(), "h": self.h.detach().cpu().clone(),
                "adam": self.adam.detach().cpu().clone(), "counter": self.counter.cpu().clone(),
                "probs": [dict(p) for p in self.probs], "opt": dict(self.opt_dict)}

    def load_state_dict(self, sd: dict):
        if [dict(p) for p in sd["probs"]] != self.probs:
            raise ValueError("checkpoint belongs to another batch")
        self.z.copy_(sd["z"].to(self.z.device))
        self.h.copy_(sd["h"].to(self.h.device))
        self.adam.copy_(sd["adam"].to(self.adam.device))
        self.counter.copy_(sd["counter"].to(self.counter.device))

    def numpy_state(self, i: int = 0) -> dict:
        """Problem i's state as float64 / complex128 arrays (oracle layout)."""
        p = self.probs[i]
        M, N, L = p["M"], p["N"], p["L"]
        z = self.batch.unpack_z(self.z, i).cpu().numpy().astype(np.float64)
        h = self.batch.unpack_w(self.h, i).cpu().numpy().astype(np.complex128)
        a = self.batch.unpack_adam(self.adam, i).cpu().numpy().astype(np.float64)
        mnl = M * N * L
        state = {"mz": a[:mnl].reshape(M, N, L), "vz": a[mnl:2 * mnl].reshape(M, N, L),
                 "mh": a[2 * mnl: 2 * mnl + 2 * M * N].reshape(M, N, 2),
                 "vh": a[2 * mnl + 2 * M * N:].reshape(M, N, 2)}
        return {"z": z, "h": h, "state": state, "t": self.t}


class StopRule:
    """The stopping criterion of Algorithm 1, per design.

    The paper ends a run when lowering the loss no longer improves the WPSL of
    the hard-quantised design, or after T outer iterations. Read here as: at
    every checkpoint the hard WPSL (dB) is compared with the best seen so far;
    a checkpoint that does not lower it by more than `min_gain_db` counts as a
    stall, and a design stops after `patience` consecutive stalls."""

    def __init__(self, n: int, patience: int = 4, min_gain_db: float = 0.0):
        if patience < 1:
            raise ValueError("patience must be >= 1")
        self.patience = int(patience)
        self.min_gain_db = float(min_gain_db)
        self.best = np.full(n, np.inf)
        self.stall = np.zeros(n, dtype=np.int64)
        self.stopped = np.zeros(n, dtype=bool)

    def update(self, ids, wpsl_db) -> list:
        """Record the checkpoint WPSL of the running designs `ids`; returns the
        ids that stop at this checkpoint."""
        out = []
        for i, w in zip(ids, wpsl_db):
            if self.stopped[i]:
                raise ValueError(f"design {i} has already stopped")
            if w < self.best[i] - self.min_gain_db:
                self.best[i] = w
                self.stall[i] = 0
            else:
                self.stall[i] += 1
                if self.stall[i] >= self.patience:
                    self.stopped[i] = True
                    out.append(int(i))
        return out


def optimise(probs, opt: dict, seeds=None, z0=None, max_iters: int | None = None, check_every: int = 50,
             patience: int = 4, min_gain_db: float = 0.0, iters_per_graph: int = 10, schedule=None) -> dict:
    """Algorithm 1 for a batch of designs, with its stopping criterion.

    Every `check_every` outer iterations the hard-quantised WPSL of each running
    design is measured (one forward evaluation of the batch) and fed to a
    StopRule; a design that stops keeps the state it has at that checkpoint,
    and the running designs continue as a smaller batch (SQNGD.subset), so
    stopped designs cost nothing further. Returns, per design, the iteration at
    which it stopped (max_iters if it never did), its hard phase indices,
    filters, logits, final hard statistics and its WPSL history."""
    max_iters = int(opt["total_iters"] if max_iters is None else max_iters)
    run = SQNGD(probs, opt, seeds=seeds, z0=z0, schedule=schedule)
    n = run.batch.n
    rule = StopRule(n, patience, min_gain_db)
    ids = list(range(n))  # original index of each problem of `run`
    res = [None] * n
    hist = [[] for _ in range(n)]
    it = 0
    while ids:
        k = min(check_every, max_iters - it)
        if k > 0:
            run.run(k, use_graph=True, iters_per_graph=min(iters_per_graph, k))
            it += k
        sts = run.hard_stats()
        for j, st in enumerate(sts):
            hist[ids[j]].append(st["pslr_db"])
        stopping = set(rule.update(ids, [st["pslr_db"] for st in sts]))
        if it >= max_iters:
            stopping = set(ids)
        if not stopping:
            continue
        idx_all = run.hard_indices()
        keep = []
        for j, i in enumerate(ids):
            if i in stopping:
                res[i] = {"stop_iter": it, "stats": sts[j], "idx": idx_all[j],
                          "h": run.batch.unpack_w(run.h, j).cpu().numpy(),
                          "z": run.batch.unpack_z(run.z, j).cpu().numpy()}
            else:
                keep.append(j)
        if keep:
            run = run.subset(keep)
        ids = [ids[j] for j in keep]
    for i in range(n):
        res[i]["wpsl_db_history"] = hist[i]
    return {"designs": res, "check_every": check_every, "patience": patience, "max_iters": max_iters}


def optimise_on_device(probs, opt: dict, seeds=None, z0=None, max_iters: int | None = None, check_every: int = 50,
                       patience: int = 4, min_gain_db: float = 0.0, poll_every: int = 4, schedule=None) -> dict:
    """Algorithm 1 for a batch of designs with its stopping criterion applied
    on the device (sqngd_stop_update + the stop mask of sqngd_set_stop_mask):
    one HIP graph per checkpoint holds `check_every` outer iterations, the
    hard-waveform evaluation of the batch and the stop update, so no host
    round trip decides anything. A stopped design keeps the state it had at
    its stopping checkpoint (its updates are masked) while the others go on in
    the same batch. The host reads the stop flags every `poll_every`
    checkpoints and ends the run once every design has stopped or `max_iters`
    outer iterations are done. The decisions equal StopRule's on the same
    checkpoint statistics. Returns, per design, the iteration at which it
    stopped (max_iters if it never did), its hard phase indices, filters,
    logits and hard statistics at the end."""
    max_iters = int(opt["total_iters"] if max_iters is None else max_iters)
    if check_every < 1 or max_iters % check_every != 0:
        raise ValueError("max_iters must be a positive multiple of check_every")
    run = SQNGD(probs, opt, seeds=seeds, z0=z0, schedule=schedule)
    n = run.batch.n
    dev = run.batch.device
    best = torch.full((n,), float("inf"), dtype=torch.float32, device=dev)
    stall = torch.zeros(n, dtype=torch.int32, device=dev)
    stopped = torch.zeros(n, dtype=torch.int32, device=dev)
    stop_iter = torch.full((n,), max_iters, dtype=torch.int32, device=dev)
    hard = run.batch.new_stats()
    run.batch.set_stop_mask(stopped)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run.step(check_every)
        run.batch.af_forward(run.z, run.h, nat.WAVE_HARD, stats=hard)
        nat.stop_update(hard, min_gain_db, patience, run.counter, best, stall, stopped, stop_iter)
    it = 0
    checks = 0
    while it < max_iters:
        g.replay()
        it += check_every
        checks += 1
        if checks % poll_every == 0 and bool(stopped.all().item()):
            break
    torch.cuda.synchronize()
    sts = nat.decode_stats(hard.cpu().numpy())
    idx = run.hard_indices()
    res = []
    for j in range(n):
        res.append({"stop_iter": int(stop_iter[j].item()), "stopped": bool(stopped[j].item()), "stats": sts[j],
                    "idx": idx[j], "h": run.batch.unpack_w(run.h, j).cpu().numpy(),
                    "z": run.batch.unpack_z(run.z, j).cpu().numpy()})
    return {"designs": res, "check_every": check_every, "patience": patience, "max_iters": max_iters,
            "iterations_run": it, "run": run}

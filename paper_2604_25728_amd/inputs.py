"""Seeded synthetic inputs and the workload presets.

This module holds no arithmetic of the method: it only draws random numbers
and states shapes and hyper-parameters. Both the GPU path and the oracle take
their inputs from here.

Workloads. The paper uses no dataset: its designs start from random phases
(Algorithm 1, initialisation). The presets below are the five workloads this
implementation is measured and checked on:

  small_m2n64   M=2, N=64, L=4, F=33 over nu in [-0.5, 0.5], p=8, 200
                iterations at step 1e-2, temperature 1.0 (small enough for
                the oracle to run whole);
  m4n256        M=4, N=256, L=8, F=129 over [-0.5, 0.5], p=16, SNRL target
                0.5 dB, temperature annealed 1.0 -> 0.05 over 2000
                iterations, step 1e-2;
  uneven        (uneven_designs) 64 designs with N in {128, 256, 512, 1024},
                M in {2, 4, 8}, L in {4, 8, 16}, F=129, 8 random restarts
                each, the m4n256 schedule;
  wide_m8n1024  M=8, N=1024, L=16, F=257 over the wide span [-2.5, 2.5],
                p=16, 5000 iterations;
  m4n512        M=4, N=512, L=8, F=129 over [-0.5, 0.5], p=16;
  m4n512_ws     the same design size with eps = 0.1 (w_psl 0.1, w_snrl 0.9)
                and SNRL target 0.3 dB: the warm-start network's workload.

Every delay is in the region of interest, SNRL target 0.5 dB, loss weights
w_psl = w_snrl = 1, Adam with beta = (0.9, 0.999), eps = 1e-8 and one step A
plus one step B per outer iteration, unless a preset says otherwise.
"""
from __future__ import annotations

import copy

import numpy as np

PHASE_MEAN = 0
PHASOR_MEAN = 1


def make_problem(M: int, N: int, L: int, F: int, nu_min: float = -0.5, nu_max: float = 0.5,
                 p: float = 16.0, snrl_target_db: float = 0.5, w_psl: float = 1.0,
                 w_snrl: float = 1.0, temperature: float = 1.0, sq_mode: int = PHASE_MEAN,
                 tau_lo: int | None = None, tau_hi: int | None = None, auto_mask: int = 0) -> dict:
    """A problem dict with every delay in the region of interest by default.

    auto_mask 0 leaves every auto pair's tau = 0 cut out of the region (eq. 8),
    1 only its Doppler-mainlobe cells |nu_f| < 1."""
    return {
        "M": int(M), "N": int(N), "L": int(L), "F": int(F),
        "nu_min": float(nu_min), "nu_max": float(nu_max),
        "tau_lo": int(-(N - 1) if tau_lo is None else tau_lo),
        "tau_hi": int((N - 1) if tau_hi is None else tau_hi),
        "p": float(p), "snrl_target_db": float(snrl_target_db),
        "w_psl": float(w_psl), "w_snrl": float(w_snrl),
        "temperature": float(temperature), "sq_mode": int(sq_mode),
        "auto_mask": int(auto_mask),
    }


def make_opt(lr_z: float = 1e-2, lr_h: float = 1e-2, beta1: float = 0.9, beta2: float = 0.999,
             eps: float = 1e-8, n_h: int = 1, n_x: int = 1, T0: float = 1.0, T1: float = 1.0,
             total_iters: int = 1, flags: int = 0) -> dict:
    return {"lr_z": float(lr_z), "lr_h": float(lr_h), "beta1": float(beta1),
            "beta2": float(beta2), "eps": float(eps), "n_h": int(n_h), "n_x": int(n_x),
            "T0": float(T0), "T1": float(T1), "total_iters": int(total_iters),
            "flags": int(flags)}


CONFIGS = {
    "m2n64": {"problem": make_problem(2, 64, 4, 33, p=8.0),
           "opt": make_opt(total_iters=200, T0=1.0, T1=1.0)},
    "m4n256": {"problem": make_problem(4, 256, 8, 129, p=16.0),
           "opt": make_opt(total_iters=2000, T0=1.0, T1=0.05)},
    "wide_m8n1024": {"problem": make_problem(8, 1024, 16, 257, nu_min=-2.5, nu_max=2.5, p=16.0),
           "opt": make_opt(total_iters=5000, T0=1.0, T1=0.05)},
    "m4n512": {"problem": make_problem(4, 512, 8, 129, p=16.0),
           "opt": make_opt(total_iters=2000, T0=1.0, T1=0.05)},
    # the warm-start workload: the paper's weighting eps = 0.1 (w_psl 0.1,
    # w_snrl 0.9) with the SNRL target 0.2 dB inside the 0.5 dB bound the
    # comparison is held to (the penalty's equilibrium sits past its target
    # while the sidelobe term pulls against it)
    "m4n512_ws": {"problem": make_problem(4, 512, 8, 129, p=16.0, w_psl=0.1, w_snrl=0.9, snrl_target_db=0.3),
           "opt": make_opt(total_iters=2000, T0=1.0, T1=0.05)},
}


def config(name: str) -> dict:
    """A deep copy of a preset: {"problem": ..., "opt": ...}."""
    return copy.deepcopy(CONFIGS[name])


def uneven_designs(n_designs: int = 64, restarts: int = 8, draw_seed: int = 12345):
    """The uneven batch: (problem, seed) for every design and restart. Shapes
    come from their own generator; restart r of design d uses seed 1000 d + r."""
    rng = np.random.default_rng(draw_seed)
    out = []
    for d in range(n_designs):
        N = int(rng.choice([128, 256, 512, 1024]))
        M = int(rng.choice([2, 4, 8]))
        L = int(rng.choice([4, 8, 16]))
        prob = make_problem(M, N, L, 129, p=16.0)
        for r in range(restarts):
            out.append((prob, 1000 * d + r))
    return out


def logits(M: int, N: int, L: int, seed: int) -> np.ndarray:
    """z ~ N(0, 1) i.i.d., drawn in float64 in [M][N][L] order, rounded to float32."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((M, N, L)).astype(np.float32)


def complex_gaussian(M: int, N: int, seed: int) -> np.ndarray:
    """A complex [M][N] sequence with i.i.d. N(0, 1/2) parts, rounded to complex64."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((M, N, 2)) * np.sqrt(0.5)
    return (a[..., 0] + 1j * a[..., 1]).astype(np.complex64)


def unimodular(M: int, N: int, seed: int) -> np.ndarray:
    """Random continuous phases e^{j 2 pi u}, u ~ U[0, 1), rounded to complex64."""
    rng = np.random.default_rng(seed)
    return np.exp(2j * np.pi * rng.random((M, N))).astype(np.complex64)


def roi_weights(prob: dict, seed: int, lo: float = 0.25, hi: float = 2.0) -> np.ndarray:
    """Weights w(tau, f) of eq. 8-9 for a problem: i.i.d. U[lo, hi) as float32
    [F][2N-1] (tau + N - 1 fastest), so that every cell of the delay-Doppler
    grid carries its own weight."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(prob["F"], 2 * prob["N"] - 1)).astype(np.float32)


def roi_window_weights(prob: dict, half_width: int) -> np.ndarray:
    """0/1 weights of a delay window |tau| <= half_width at every Doppler bin
    (the paper's fixed ROI tau in [-50, 50] is half_width = 50), float32 [F][2N-1]."""
    tau = np.arange(-(prob["N"] - 1), prob["N"])
    return np.tile((np.abs(tau) <= half_width).astype(np.float32), (prob["F"], 1))


def noise(M: int, N: int, seed: int) -> np.ndarray:
    """The warm-start network's input noise, N(0, 1) [M][N] float32."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((M, N)).astype(np.float32)


# ---------------------------------------------------------------- warm-start network

NET_CHANNELS = 64   # hidden channels
NET_TAPS = 5        # kernel width (zero padding of 2 on each side, output length N)


def net_layers(M: int, L: int) -> list:
    """(input channels, output channels) of the four conv layers: M noise rows
    plus two conditioning rows in, 64 hidden channels, M*L logits out (channel
    m*L + l is level l of waveform m)."""
    C = NET_CHANNELS
    return [(M + 2, C), (C, C), (C, C), (C, M * L)]


def net_param_count(M: int, L: int) -> int:
    return sum(co * NET_TAPS * ci + co for ci, co in net_layers(M, L))


def net_init(M: int, L: int, seed: int) -> np.ndarray:
    """Flat float32 parameters, per layer W[cout][tap][cin] then b[cout]:
    uniform in +-sqrt(6 / fan_in) for W (fan_in = 5 cin), zero bias."""
    rng = np.random.default_rng(seed)
    out = []
    for ci, co in net_layers(M, L):
        bound = np.sqrt(6.0 / (NET_TAPS * ci))
        out.append(rng.uniform(-bound, bound, size=co * NET_TAPS * ci))
        out.append(np.zeros(co))
    return np.concatenate(out).astype(np.float32)


def net_noise(B: int, M: int, N: int, seed: int) -> np.ndarray:
    """A batch of network inputs, N(0, 1) [B][M][N] float32."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((B, M, N)).astype(np.float32)


def net_targets(B: int, M: int, N: int, L: int, seed: int) -> np.ndarray:
    """Random level indices [B][M][N] int32 (for tests of the loss)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, L, size=(B, M, N)).astype(np.int32)


# ------------------------------------- the paper's transmit network (Sec. III-A)

SQN_WIDTH = 128     # hidden width of the ResNet
SQN_BLOCKS = 5      # residual blocks


def sqn_layers(D: int) -> list:
    """(input, output) widths of the dense layers, in parameter order: the input
    layer, two per residual block, the output layer (D = M N inputs and outputs)."""
    H = SQN_WIDTH
    return [(D, H)] + [(H, H)] * (2 * SQN_BLOCKS) + [(H, D)]


def sqn_param_count(D: int) -> int:
    return sum(o * i + o for i, o in sqn_layers(D))


def sqn_init(D: int, seed: int) -> np.ndarray:
    """Flat float32 parameters, per layer W[out][in] then b[out], uniform in
    +-1/sqrt(in) (weights and biases)."""
    rng = np.random.default_rng(seed)
    out = []
    for i, o in sqn_layers(D):
        bound = 1.0 / np.sqrt(i)
        out.append(rng.uniform(-bound, bound, size=o * i))
        out.append(rng.uniform(-bound, bound, size=o))
    return np.concatenate(out).astype(np.float32)


def sqn_thresholds(B: int, copies: int) -> np.ndarray:
    """The B * copies ordered thresholds rho_i = (i + 1/2) / (B copies) of the
    copied staircase, float32."""
    K = B * copies
    return ((np.arange(K) + 0.5) / K).astype(np.float32)


def sqn_input(M: int, N: int, B: int, seed: int) -> np.ndarray:
    """The network input y0 = vec(Y0) of Algorithm 1's initialisation: random
    normalised discrete phases b / B, b uniform in [0, B), float32 [M N]
    (waveform m's chips at m N .. m N + N - 1, the column-stacking of the
    N x M phase matrix)."""
    rng = np.random.default_rng(seed)
    return (rng.integers(0, B, size=M * N) / B).astype(np.float32)

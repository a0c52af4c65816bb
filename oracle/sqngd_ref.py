"""FP64 CPU oracle of the SQNGD hot path (arXiv 2604.25728).

TEST INFRASTRUCTURE ONLY: the correctness reference for the gfx950 kernels.
Only the tests, the package smoke check and the CPU-baseline leg of the
benchmark may import it. It shares no code with the HIP path and never
imports the product package.

The heavy sums (the ambiguity function of eq. 6, the loss of eq. 7-10 and
37-42, their gradients) are direct sums in ``af_oracle.c``; this module adds
the transmit parameterisation, the optimiser and one outer iteration of
Algorithm 1, all in float64 with numpy.

Readings of the paper used throughout (each listed with its reason in the
design notes of the repository):
  * indices are 0-based (the paper counts from 1; |A| is unchanged);
  * the Doppler grid is uniform and includes both end points;
  * the transmit side is L real logits per chip; the soft waveform is the
    phase-mean exp(j 2 pi sum_l l softmax(z/T)_l / L) (unimodular, like the
    soft waveform of eq. 23), the hard waveform exp(j 2 pi argmax(z) / L);
  * the matched-filter start is h0 = x0 (so that h^H x = N and the SNRL is
    0 dB), not the conjugate written in eq. 30;
  * the max of eq. 37 is replaced by a p-norm over the union of auto and
    cross sidelobe cells, with a = |A| / N;
  * gradients of the real loss with respect to a complex variable v are packed
    as dL/dRe(v) + j dL/dIm(v).

A problem is a plain dict with the keys M, N, L, F, nu_min, nu_max, tau_lo,
tau_hi, p, snrl_target_db, w_psl, w_snrl, temperature, sq_mode (0 phase-mean,
1 phasor-mean), optionally auto_mask (0, the default: an auto pair's whole
tau = 0 cut is outside the region, eq. 8; 1: only its Doppler-mainlobe cells
|nu_f| < 1 are) and optionally roi_w: the weights w(tau, f) of eq. 8-9 as an
[F][2N-1] array (tau + N - 1 fastest; absent or None means w = 1). Options of an outer iteration are a dict with lr_z, lr_h,
beta1, beta2, eps, n_h, n_x, T0, T1, total_iters, flags (1 = plain gradient
descent).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "af_oracle.c")
_SO = os.path.join(_HERE, "libsqngd_oracle.so")
_lib = None

PHASE_MEAN = 0
PHASOR_MEAN = 1
OPT_SGD = 1


def build(force: bool = False) -> str:
    """Compile af_oracle.c with gcc (FP64, OpenMP) into libsqngd_oracle.so."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-fopenmp", "-fcx-limited-range", "-fPIC", "-shared", "-std=c11",
               _SRC, "-o", _SO, "-lm"]
        subprocess.run(cmd, check=True)
    return _SO


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        d, i, P = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        lib.sqngd_ref_nu.restype = d
        lib.sqngd_ref_nu.argtypes = [i, d, d, i]
        lib.sqngd_ref_af_cube.restype = None
        lib.sqngd_ref_af_cube.argtypes = [i, i, i, d, d, P, P, P]
        lib.sqngd_ref_af_row.restype = None
        lib.sqngd_ref_af_row.argtypes = [i, i, i, d, d, P, P, i, i, i, P]
        lib.sqngd_ref_loss.restype = None
        lib.sqngd_ref_loss.argtypes = [i, i, i, d, d, P, P, P, i, i, i, P, d, d, d, d, P, P, P, P]
        lib.sqngd_ref_grads.restype = None
        lib.sqngd_ref_grads.argtypes = [i, i, i, d, d, P, P, P, i, i, i, P, d, d, d, d, P, P]
        _lib = lib
    return _lib


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# Ambiguity function and loss (Sec. II-A and Sec. III-B)
# ---------------------------------------------------------------------------

def doppler_grid(F: int, nu_min: float, nu_max: float) -> np.ndarray:
    """Doppler bins nu_f, f = 0..F-1 (uniform, both end points included)."""
    lib = _load()
    return np.array([lib.sqngd_ref_nu(int(F), float(nu_min), float(nu_max), f) for f in range(F)])


def af_cube(s, h, F: int, nu_min: float, nu_max: float) -> np.ndarray:
    """A[m][l][f][tau + N - 1] = sum_n s_m(n) e^{j2 pi n nu_f/N} conj(h_l(n + tau)) (eq. 6)."""
    s, h = _c128(s), _c128(h)
    M, N = s.shape
    assert h.shape == (M, N)
    out = np.zeros((M, M, F, 2 * N - 1), dtype=np.complex128)
    _load().sqngd_ref_af_cube(M, N, F, float(nu_min), float(nu_max), _ptr(s), _ptr(h), _ptr(out))
    return out


def af_row(s, h, F: int, nu_min: float, nu_max: float, m: int, l: int, f: int) -> np.ndarray:
    """One row A_ml(., f) of the cube (eq. 6), for sampled checks."""
    s, h = _c128(s), _c128(h)
    M, N = s.shape
    out = np.zeros(2 * N - 1, dtype=np.complex128)
    _load().sqngd_ref_af_row(M, N, F, float(nu_min), float(nu_max), _ptr(s), _ptr(h), m, l, f,
                             _ptr(out))
    return out


def _weights(prob: dict, N: int, F: int):
    """The weight table w(tau, f) of eq. 8-9 as contiguous float64 [F][2N-1], or None."""
    wt = prob.get("roi_w")
    if wt is None:
        return None
    wt = np.ascontiguousarray(wt, dtype=np.float64)
    assert wt.shape == (F, 2 * N - 1), wt.shape
    return wt


def loss_stats(cube: np.ndarray, s, h, prob: dict) -> dict:
    """Loss, p-norm, SNRL penalty, PSLs and SNRLs of one evaluation (eq. 7-10, 37-42, 48)."""
    s, h = _c128(s), _c128(h)
    cube = _c128(cube)
    M, N = s.shape
    F = cube.shape[2]
    out = np.zeros(8)
    arg = np.zeros(4, dtype=np.int32)
    snrl = np.zeros(M)
    pm = np.zeros(M)
    wt = _weights(prob, N, F)
    _load().sqngd_ref_loss(M, N, F, float(prob["nu_min"]), float(prob["nu_max"]), _ptr(cube), _ptr(s),
                           _ptr(h), int(prob["tau_lo"]), int(prob["tau_hi"]), int(prob.get("auto_mask", 0)),
                           _ptr(wt), float(prob["p"]), float(prob["snrl_target_db"]),
                           float(prob["w_psl"]), float(prob["w_snrl"]), _ptr(out), _ptr(arg),
                           _ptr(snrl), _ptr(pm))
    keys = ["loss", "lp", "l_snrl", "psl_auto", "psl_cross", "pslr_db", "snrl_db_max", "p_min"]
    st = {k: float(v) for k, v in zip(keys, out)}
    st["arg"] = tuple(int(v) for v in arg)
    st["snrl_db"] = snrl
    st["p_m"] = pm
    return st


def grads(s, h, prob: dict, cube: np.ndarray | None = None):
    """Packed gradients (grad_s, grad_h) of the loss of loss_stats (direct sums)."""
    s, h = _c128(s), _c128(h)
    M, N = s.shape
    F = int(prob["F"])
    if cube is None:
        cube = af_cube(s, h, F, prob["nu_min"], prob["nu_max"])
    cube = _c128(cube)
    gs = np.zeros((M, N), dtype=np.complex128)
    gh = np.zeros((M, N), dtype=np.complex128)
    wt = _weights(prob, N, F)
    _load().sqngd_ref_grads(M, N, F, float(prob["nu_min"]), float(prob["nu_max"]), _ptr(s), _ptr(h),
                            _ptr(cube), int(prob["tau_lo"]), int(prob["tau_hi"]), int(prob.get("auto_mask", 0)),
                            _ptr(wt), float(prob["p"]),
                            float(prob["snrl_target_db"]), float(prob["w_psl"]),
                            float(prob["w_snrl"]), _ptr(gs), _ptr(gh))
    return gs, gh


def evaluate(s, h, prob: dict, want_grads: bool = True):
    """Stats and (optionally) packed gradients of one evaluation."""
    cube = af_cube(s, h, int(prob["F"]), prob["nu_min"], prob["nu_max"])
    st = loss_stats(cube, s, h, prob)
    if not want_grads:
        return st, None, None
    gs, gh = grads(s, h, prob, cube)
    return st, gs, gh


# ---------------------------------------------------------------------------
# Transmit parameterisation (the analog of Sec. III-A, eq. 18-23)
# ---------------------------------------------------------------------------

def softmax(z, T: float) -> np.ndarray:
    """softmax over the last axis of z / T, with the maximum subtracted."""
    a = np.asarray(z, dtype=np.float64) / float(T)
    a = a - a.max(axis=-1, keepdims=True)
    e = np.exp(a)
    return e / e.sum(axis=-1, keepdims=True)


def soft_waveform(z, T: float, mode: int = PHASE_MEAN) -> np.ndarray:
    """Soft-quantised waveform [M][N] from logits [M][N][L] at temperature T."""
    z = np.asarray(z, dtype=np.float64)
    L = z.shape[-1]
    pi = softmax(z, T)
    levels = np.arange(L, dtype=np.float64)
    if mode == PHASE_MEAN:
        ybar = (pi * levels).sum(axis=-1)
        return np.exp(1j * 2.0 * np.pi * ybar / L)
    if mode == PHASOR_MEAN:
        return (pi * np.exp(1j * 2.0 * np.pi * levels / L)).sum(axis=-1)
    raise ValueError("unknown soft-quantiser mode")


def hard_indices(z) -> np.ndarray:
    """l* = argmax_l z[m][n][l], the lowest l on ties (eq. 18 analog)."""
    z = np.asarray(z)
    L = z.shape[-1]
    idx = np.full(z.shape[:-1], 0, dtype=np.int32)
    best = z[..., 0].copy()
    for l in range(1, L):
        better = z[..., l] > best
        idx[better] = l
        best = np.where(better, z[..., l], best)
    return idx


def hard_waveform(z) -> np.ndarray:
    """x = exp(j 2 pi l* / L), a point of the discrete-phase set of eq. 5."""
    z = np.asarray(z)
    L = z.shape[-1]
    return np.exp(1j * 2.0 * np.pi * hard_indices(z).astype(np.float64) / L)


def logit_grad(z, T: float, grad_s, mode: int = PHASE_MEAN) -> np.ndarray:
    """dL/dz from the packed waveform gradient grad_s by the chain rule.

    Phase-mean: s = e^{j phi}, phi = 2 pi ybar / L, ybar = sum_l l pi_l, so
    dL/dphi = Im(grad_s conj(s)) and dybar/dz_k = pi_k (k - ybar) / T.
    Phasor-mean: ds/dz_k = pi_k (u_k - s) / T with u_k = e^{j 2 pi k / L}, so
    dL/dz_k = Re(conj(grad_s) pi_k (u_k - s)) / T."""
    z = np.asarray(z, dtype=np.float64)
    L = z.shape[-1]
    pi = softmax(z, T)
    levels = np.arange(L, dtype=np.float64)
    g = np.asarray(grad_s, dtype=np.complex128)
    if mode == PHASE_MEAN:
        ybar = (pi * levels).sum(axis=-1)
        s = np.exp(1j * 2.0 * np.pi * ybar / L)
        dphi = np.imag(g * np.conj(s))
        return (dphi * 2.0 * np.pi / L)[..., None] * pi * (levels - ybar[..., None]) / T
    if mode == PHASOR_MEAN:
        u = np.exp(1j * 2.0 * np.pi * levels / L)
        s = (pi * u).sum(axis=-1)
        return np.real(np.conj(g)[..., None] * pi * (u - s[..., None])) / T
    raise ValueError("unknown soft-quantiser mode")


# ---------------------------------------------------------------------------
# Optimiser (Sec. III-A eq. 29-32, Sec. III-C, Algorithm 1)
# ---------------------------------------------------------------------------

def temperature(t: int, T0: float, T1: float, total_iters: int) -> float:
    """Geometric anneal T_t = T0 (T1/T0)^(t/(I-1)), held at T1 after the last iteration."""
    if total_iters <= 1:
        return float(T0)
    frac = min(float(t), float(total_iters - 1)) / float(total_iters - 1)
    return float(T0) * (float(T1) / float(T0)) ** frac


def adam(param, grad, m, v, t: int, lr: float, beta1: float, beta2: float, eps: float):
    """One bias-corrected Adam update of a real array (Kingma and Ba); returns new (param, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return param - lr * mhat / (np.sqrt(vhat) + eps), m, v


def project(h) -> np.ndarray:
    """Energy projection of eq. 32: h_m <- h_m sqrt(N / |h_m|^2), row by row."""
    h = np.asarray(h, dtype=np.complex128)
    N = h.shape[-1]
    e = (np.abs(h) ** 2).sum(axis=-1, keepdims=True)
    return h * np.sqrt(N / e)


def matched_init(z) -> np.ndarray:
    """Filters of Algorithm 1's initialisation: the matched filter of the hard
    starting waveform, projected (eq. 29-32, with h0 = x0)."""
    return project(hard_waveform(z))


def _c2r(c):
    c = np.asarray(c, dtype=np.complex128)
    return np.stack([c.real, c.imag], axis=-1)


def _r2c(r):
    return r[..., 0] + 1j * r[..., 1]


def new_state(M: int, N: int, L: int) -> dict:
    """Adam moments: z (m, v) [M][N][L] and h (m, v) [M][N][2] (Re, Im)."""
    return {"mz": np.zeros((M, N, L)), "vz": np.zeros((M, N, L)),
            "mh": np.zeros((M, N, 2)), "vh": np.zeros((M, N, 2))}


def step(prob: dict, opt: dict, z, h, state: dict, t: int):
    """One outer iteration t of Algorithm 1 with the logit parameterisation.

    Step A (n_h times): hard waveform from z, loss and grad_h, Adam on
    (Re h, Im h), energy projection. Step B (n_x times): soft waveform at T_t,
    loss and grad_z, Adam on z. An evaluation whose loss or gradient is not
    finite leaves the parameters unchanged. Returns (z, h, state, stats_A,
    stats_B) with the stats of the last evaluation of each step (None if the
    step did not run)."""
    z = np.array(z, dtype=np.float64)
    h = np.array(h, dtype=np.complex128)
    state = {k: np.array(v) for k, v in state.items()}
    sgd = bool(int(opt.get("flags", 0)) & OPT_SGD)
    b1, b2, eps = float(opt["beta1"]), float(opt["beta2"]), float(opt["eps"])
    stats_a = stats_b = None
    for i in range(int(opt["n_h"])):
        x = hard_waveform(z)
        stats_a, _, gh = evaluate(x, h, prob)
        if not (np.isfinite(stats_a["loss"]) and np.all(np.isfinite(gh))):
            continue
        if sgd:
            h = h - float(opt["lr_h"]) * gh
        else:
            k = t * int(opt["n_h"]) + i + 1
            hr, state["mh"], state["vh"] = adam(_c2r(h), _c2r(gh), state["mh"], state["vh"], k,
                                                float(opt["lr_h"]), b1, b2, eps)
            h = _r2c(hr)
        h = project(h)
    T = temperature(t, float(opt["T0"]), float(opt["T1"]), int(opt["total_iters"]))
    for j in range(int(opt["n_x"])):
        s = soft_waveform(z, T, int(prob.get("sq_mode", PHASE_MEAN)))
        stats_b, gs, _ = evaluate(s, h, prob)
        gz = logit_grad(z, T, gs, int(prob.get("sq_mode", PHASE_MEAN)))
        if not (np.isfinite(stats_b["loss"]) and np.all(np.isfinite(gz))):
            continue
        if sgd:
            z = z - float(opt["lr_z"]) * gz
        else:
            k = t * int(opt["n_x"]) + j + 1
            z, state["mz"], state["vz"] = adam(z, gz, state["mz"], state["vz"], k,
                                               float(opt["lr_z"]), b1, b2, eps)
    return z, h, state, stats_a, stats_b

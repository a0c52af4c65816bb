"""FP64 CPU oracle of the paper's transmit parameterisation (Sec. III-A).

TEST INFRASTRUCTURE ONLY: the correctness reference for the gfx950 kernels of
the SQN transmit side. Only the tests, the package smoke check and the
CPU-baseline leg of the benchmark may import it. It shares no code with the
HIP path.

The paper generates continuous variables z = f_theta(y0) (eq. 17) from the
fixed input y0 = vec(Y0) of random normalised discrete phases b / B (eq. 15-16,
Algorithm 1's initialisation) with a ResNet
of 5 residual blocks, width 128, tanh in the hidden and residual layers and a
sigmoid output (Sec. IV). Read here as
  h_0 = tanh(W_in y0 + b_in),
  h_k = h_{k-1} + tanh(W2_k tanh(W1_k h_{k-1} + b1_k) + b2_k),  k = 1..5,
  z   = sigmoid(W_out h_5 + b_out).
The soft quantiser is the copied tanh staircase of eq. 24 with K = B r_n
ordered thresholds rho_i and a_i = 1 / (2B) (each transition adds one level
1/B, so the hard values are the k / B of the paper's example):
  y1 = Q_A(z) = sum_i a (tanh(c (z - rho_i)) + 1),  x = exp(j 2 pi y1) (eq. 22-23).
The hard quantiser Q_R (eq. 43) is read as the staircase's limit: the number of
thresholds at or below z, divided by B (phase index = that count mod B).
After each transmit update the thresholds are sorted (the projection onto an
ordered set Sec. III-C asks for after each transmit-side update).
"""
from __future__ import annotations

import numpy as np

H = 128
BLOCKS = 5


def layers(D: int) -> list:
    return [(D, H)] + [(H, H)] * (2 * BLOCKS) + [(H, D)]


def unpack(theta, D: int) -> list:
    """[(W [out][in], b [out]), ...] in layer order, float64."""
    theta = np.asarray(theta, dtype=np.float64)
    out, off = [], 0
    for i, o in layers(D):
        W = theta[off: off + o * i].reshape(o, i)
        off += o * i
        b = theta[off: off + o]
        off += o
        out.append((W, b))
    assert off == theta.size
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in parts])


def forward(theta, y0) -> tuple:
    """z = f_theta(y0) and the values the backward pass needs."""
    y0 = np.asarray(y0, dtype=np.float64)
    D = y0.size
    P = unpack(theta, D)
    W, b = P[0]
    h = np.tanh(W @ y0 + b)
    hs, us = [h], []
    for k in range(BLOCKS):
        W1, b1 = P[1 + 2 * k]
        W2, b2 = P[2 + 2 * k]
        u = np.tanh(W1 @ h + b1)
        v = np.tanh(W2 @ u + b2)
        h = h + v
        us.append((u, v))
        hs.append(h)
    Wo, bo = P[-1]
    z = 1.0 / (1.0 + np.exp(-(Wo @ h + bo)))
    return z, {"y0": y0, "hs": hs, "us": us, "z": z, "P": P}


def backward(cache: dict, dz) -> np.ndarray:
    """dL/dtheta (flat, the layout of forward's theta) from dL/dz."""
    P, hs, us, z = cache["P"], cache["hs"], cache["us"], cache["z"]
    grads = [None] * len(P)
    dp = np.asarray(dz, dtype=np.float64) * z * (1.0 - z)      # through the sigmoid
    Wo, _ = P[-1]
    grads[-1] = (np.outer(dp, hs[-1]), dp)
    dh = Wo.T @ dp
    for k in reversed(range(BLOCKS)):
        u, v = us[k]
        W1, _ = P[1 + 2 * k]
        W2, _ = P[2 + 2 * k]
        dv = dh * (1.0 - v * v)                                 # through tanh of the residual branch
        grads[2 + 2 * k] = (np.outer(dv, u), dv)
        du = (W2.T @ dv) * (1.0 - u * u)
        grads[1 + 2 * k] = (np.outer(du, hs[k]), du)
        dh = dh + W1.T @ du                                     # skip connection plus the branch
    h0 = hs[0]
    dp0 = dh * (1.0 - h0 * h0)
    grads[0] = (np.outer(dp0, cache["y0"]), dp0)
    return pack(grads)


def soft_quantise(z, rho, B: int, c: float) -> np.ndarray:
    """y1 = Q_A(z) (eq. 24): sum over the thresholds of a (tanh(c (z - rho_i)) + 1), a = 1/(2B)."""
    z = np.asarray(z, dtype=np.float64)
    t = np.tanh(c * (z[:, None] - np.asarray(rho, dtype=np.float64)[None, :]))
    return ((t + 1.0) / (2.0 * B)).sum(axis=1)


def sech2(x) -> np.ndarray:
    """tanh'(x) = 1 - tanh(x)^2 (the derivative the paper states for the
    staircase), evaluated as 4 e / (1 + e)^2 with e = exp(-2 |x|) so that it
    keeps its relative precision where tanh(x) rounds to +-1."""
    e = np.exp(-2.0 * np.abs(np.asarray(x, dtype=np.float64)))
    return 4.0 * e / ((1.0 + e) * (1.0 + e))


def soft_quantise_grad(z, rho, B: int, c: float, dy) -> tuple:
    """(dL/dz, dL/drho) from dL/dy1 through Q_A."""
    z = np.asarray(z, dtype=np.float64)
    d = c * sech2(c * (z[:, None] - np.asarray(rho, dtype=np.float64)[None, :])) / (2.0 * B)  # dQ_A/dz
    dy = np.asarray(dy, dtype=np.float64)
    return (dy[:, None] * d).sum(axis=1), -(dy[:, None] * d).sum(axis=0)


def hard_levels(z, rho) -> np.ndarray:
    """Number of thresholds at or below z (the hard quantiser's level count)."""
    return (np.asarray(rho, dtype=np.float64)[None, :] <= np.asarray(z, dtype=np.float64)[:, None]).sum(axis=1)


def hard_waveform(z, rho, B: int, M: int, N: int) -> tuple:
    """Phase indices (count mod B) [M][N] and x = exp(j 2 pi index / B)."""
    k = hard_levels(z, rho) % B
    return k.reshape(M, N), np.exp(2j * np.pi * k / B).reshape(M, N)


def soft_waveform(y1, M: int, N: int) -> np.ndarray:
    return np.exp(2j * np.pi * np.asarray(y1, dtype=np.float64)).reshape(M, N)


def waveform_chain(grad_s, s) -> np.ndarray:
    """dL/dy1 from the packed waveform gradient: s = exp(j 2 pi y1), so
    dL/dy1 = 2 pi Im(grad_s conj(s)), flat [M N]."""
    return (2.0 * np.pi * np.imag(np.asarray(grad_s) * np.conj(np.asarray(s)))).reshape(-1)


def initial_filters(y0, M: int, N: int) -> np.ndarray:
    """Algorithm 1's initialisation: X0 = exp(j 2 pi Y0) (eq. 29) from the
    network input y0 = vec(Y0), the filters its matched filter -- read as
    H0 = X0 (eq. 30 prints the conjugate, which under eq. 6 would not give the
    mainlobe h^H x0 = N) -- each row projected to energy N (eq. 32)."""
    x0 = np.exp(2j * np.pi * np.asarray(y0, dtype=np.float64)).reshape(M, N)
    return x0 * np.sqrt(N / (np.abs(x0) ** 2).sum(axis=1, keepdims=True))


def new_state(D: int, K: int, M: int, N: int) -> dict:
    """Adam moments of theta, rho and (Re h, Im h)."""
    P = sum(o * i + o for i, o in layers(D))
    return {"mt": np.zeros(P), "vt": np.zeros(P), "mr": np.zeros(K), "vr": np.zeros(K),
            "mh": np.zeros((M, N, 2)), "vh": np.zeros((M, N, 2))}


def iteration(prob: dict, opt: dict, sqn: dict, theta, rho, h, y0, state: dict, t: int,
              matched: bool = False):
    """One outer iteration t of Algorithm 1 with the paper's transmit side:
    step A (n_h times) on the filters with the hard waveform Q_R(f_theta(y0)),
    Adam on (Re h, Im h) with lr_h and the energy projection; step B (n_x
    times) on (theta, rho) with the soft waveform Q_A(f_theta(y0)), Adam with
    lr_z on both, then the thresholds sorted. sqn holds B (= prob["L"]),
    copies and c. Returns (theta, rho, h, state, stats_A, stats_B).

    matched=True: the AF extension of SQN that the paper compares against
    (Sec. IV) -- no step A, and in step B the filters are the soft waveform
    itself, so the waveform gradient is the sum of the gradients of L(s, h)
    in its two arguments at h = s (h is returned unchanged)."""
    from oracle import sqngd_ref as R
    M, N = prob["M"], prob["N"]
    B, c = int(prob["L"]), float(sqn["c"])
    theta = np.array(theta, dtype=np.float64)
    rho = np.array(rho, dtype=np.float64)
    h = np.array(h, dtype=np.complex128)
    state = {k: np.array(v) for k, v in state.items()}
    b1, b2, eps = float(opt["beta1"]), float(opt["beta2"]), float(opt["eps"])
    stats_a = stats_b = None
    z, _ = forward(theta, y0)
    _, x = hard_waveform(z, rho, B, M, N)
    for i in range(0 if matched else int(opt["n_h"])):
        stats_a, _, gh = R.evaluate(x, h, prob)
        k = t * int(opt["n_h"]) + i + 1
        hr, state["mh"], state["vh"] = R.adam(R._c2r(h), R._c2r(gh), state["mh"], state["vh"], k,
                                              float(opt["lr_h"]), b1, b2, eps)
        h = R.project(R._r2c(hr))
    for j in range(int(opt["n_x"])):
        z, cache = forward(theta, y0)
        s = soft_waveform(soft_quantise(z, rho, B, c), M, N)
        if matched:
            stats_b, gs, gh = R.evaluate(s, s, prob)
            gs = gs + gh
        else:
            stats_b, gs, _ = R.evaluate(s, h, prob)
        dz, drho = soft_quantise_grad(z, rho, B, c, waveform_chain(gs, s))
        dtheta = backward(cache, dz)
        k = t * int(opt["n_x"]) + j + 1
        theta, state["mt"], state["vt"] = R.adam(theta, dtheta, state["mt"], state["vt"], k,
                                                 float(opt["lr_z"]), b1, b2, eps)
        rho, state["mr"], state["vr"] = R.adam(rho, drho, state["mr"], state["vr"], k,
                                               float(opt["lr_z"]), b1, b2, eps)
        rho = np.sort(rho)
    return theta, rho, h, state, stats_a, stats_b

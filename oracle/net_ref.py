"""FP64 CPU oracle of the learned warm-start network.

TEST INFRASTRUCTURE ONLY: the correctness reference for the gfx950 network
kernels. Only the tests, the package smoke check and the CPU-baseline leg of
the benchmark may import it. It shares no code with the HIP path.

The network is not part of the paper's method (the paper reparameterises each
design with its own ResNet, Sec. III-A eq. 17, and trains it per design); it
proposes starting logits for the optimiser of Algorithm 1. It is a 1-D
convolutional net over the chip axis n:

  X0[b][n][c]  = noise[b][c][n] for c < M, cond[0], cond[1] for c = M, M+1;
  Z_i[b][n][o] = b_i[o] + sum_{tap < 5} sum_c W_i[o][tap][c] X_i[b][n + tap - 2][c]
                 (zero outside 0 <= n + tap - 2 < N);
  X_{i+1}      = relu(Z_i) for i = 0, 1, 2;   logits z[b][m][n][l] = Z_3[b][n][m L + l];
  loss         = mean over (b, m, n) of the cross-entropy of softmax_l(z[b][m][n][:])
                 against a target level t[b][m][n].

With rounding=True every value the device kernels hold in bfloat16 is rounded
to bfloat16 (round to nearest even) at the same place: the weights, the input
X0, the activations X1..X3, the logit gradient fed back and the activation
gradients dZ0..dZ2; everything else is exact FP64. With rounding=False the
whole computation is FP64.
"""
from __future__ import annotations

import numpy as np

TAPS = 5
HALF = 2


def bf16(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)


def layers(M: int, L: int, C: int = 64) -> list:
    return [(M + 2, C), (C, C), (C, C), (C, M * L)]


def unpack(params, M: int, L: int) -> list:
    """Flat parameters -> [(W[cout][tap][cin], b[cout])] in float64."""
    p = np.asarray(params, dtype=np.float64)
    out, off = [], 0
    for ci, co in layers(M, L):
        W = p[off: off + co * TAPS * ci].reshape(co, TAPS, ci)
        off += co * TAPS * ci
        b = p[off: off + co]
        off += co
        out.append((W, b))
    assert off == p.size
    return out


def pack(items) -> np.ndarray:
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in items])


def shift(X, d: int) -> np.ndarray:
    """Y[b][n] = X[b][n + d] (zero where n + d is outside [0, N))."""
    B, N, C = X.shape
    Y = np.zeros_like(X)
    if d >= 0:
        Y[:, : N - d] = X[:, d:]
    else:
        Y[:, -d:] = X[:, : N + d]
    return Y


def conv(X, W) -> np.ndarray:
    """Z[b][n][o] = sum_tap sum_c W[o][tap][c] X[b][n + tap - 2][c]."""
    Z = np.zeros(X.shape[:2] + (W.shape[0],))
    for tap in range(TAPS):
        Z += shift(X, tap - HALF) @ W[:, tap, :].T
    return Z


def conv_input_grad(dZ, W) -> np.ndarray:
    """dX[b][n][c] = sum_tap sum_o W[o][tap][c] dZ[b][n - tap + 2][o] (adjoint of conv)."""
    dX = np.zeros(dZ.shape[:2] + (W.shape[2],))
    for tap in range(TAPS):
        dX += shift(dZ, HALF - tap) @ W[:, tap, :]
    return dX


def conv_weight_grad(dZ, X) -> np.ndarray:
    """dW[o][tap][c] = sum_b sum_n dZ[b][n][o] X[b][n + tap - 2][c]."""
    B, N, Co = dZ.shape
    Ci = X.shape[2]
    dW = np.zeros((Co, TAPS, Ci))
    dz2 = dZ.reshape(B * N, Co)
    for tap in range(TAPS):
        dW[:, tap, :] = dz2.T @ shift(X, tap - HALF).reshape(B * N, Ci)
    return dW


def net_input(noise, cond) -> np.ndarray:
    noise = np.asarray(noise, dtype=np.float64)
    B, M, N = noise.shape
    X0 = np.zeros((B, N, M + 2))
    X0[:, :, :M] = noise.transpose(0, 2, 1)
    X0[:, :, M] = cond[0]
    X0[:, :, M + 1] = cond[1]
    return X0


def forward(params, noise, cond, M: int, L: int, rounding: bool = True):
    """Logits z[B][M][N][L] and the cache of the backward pass."""
    rnd = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    items = [(rnd(W), b) for W, b in unpack(params, M, L)]
    X = rnd(net_input(noise, cond))
    xs = [X]
    for i, (W, b) in enumerate(items):
        Z = conv(X, W) + b
        if i < 3:
            X = rnd(np.maximum(Z, 0.0))
            xs.append(X)
    B, N = Z.shape[:2]
    z = Z.reshape(B, N, M, L).transpose(0, 2, 1, 3).copy()
    return z, {"xs": xs, "items": items, "rounding": rounding, "M": M, "L": L}


def cross_entropy(z, target):
    """Mean cross-entropy over (b, m, n) and its gradient with respect to z."""
    z = np.asarray(z, dtype=np.float64)
    zm = z.max(axis=-1, keepdims=True)
    e = np.exp(z - zm)
    s = e.sum(axis=-1, keepdims=True)
    logp = z - zm - np.log(s)
    t = np.asarray(target)[..., None]
    cnt = t.size
    loss = -np.take_along_axis(logp, t, axis=-1).sum() / cnt
    dz = e / s
    np.put_along_axis(dz, t, np.take_along_axis(dz, t, axis=-1) - 1.0, axis=-1)
    return loss, dz / cnt


def backward(cache, dz) -> np.ndarray:
    """Gradient of a loss with respect to the flat parameters, given dL/dz."""
    rnd = bf16 if cache["rounding"] else (lambda a: np.asarray(a, dtype=np.float64))
    M, L = cache["M"], cache["L"]
    xs, items = cache["xs"], cache["items"]
    B, _, N, _ = dz.shape
    dZ = rnd(np.asarray(dz, dtype=np.float64).transpose(0, 2, 1, 3).reshape(B, N, M * L))
    grads = [None] * 4
    for i in range(3, -1, -1):
        W, _ = items[i]
        grads[i] = (conv_weight_grad(dZ, xs[i]), dZ.sum(axis=(0, 1)))
        if i > 0:
            dZ = rnd(conv_input_grad(dZ, W) * (xs[i] > 0))
    return pack(grads)

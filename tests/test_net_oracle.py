"""Pins of the warm-start network oracle (CPU): each check goes through a route
other than the oracle's own formulas (numpy.correlate, torch float64 autograd,
central differences, torch's bfloat16 conversion)."""
import numpy as np
import pytest

from oracle import net_ref as R
from paper_2604_25728_amd import inputs as I

torch = pytest.importorskip("torch")


def _small(seed=0, B=2, M=2, N=12, L=8):
    params = I.net_init(M, L, seed)
    noise = I.net_noise(B, M, N, seed + 1)
    cond = (L / 8.0, 1.0)
    return params, noise, cond, B, M, N, L


def test_bf16_rounding_matches_torch():
    x = np.random.default_rng(0).standard_normal(20000) * np.logspace(-20, 20, 20000)
    x = np.concatenate([x, [0.0, 1.0, -1.0, 1.00390625, 1.01171875, 3.0e38]])  # ties and a large value
    want = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(R.bf16(x), want)


def test_conv_is_numpy_correlate():
    rng = np.random.default_rng(1)
    B, N, Ci, Co = 2, 9, 3, 4
    X = rng.standard_normal((B, N, Ci))
    W = rng.standard_normal((Co, 5, Ci))
    Z = R.conv(X, W)
    for b in range(B):
        for o in range(Co):
            acc = np.zeros(N)
            for c in range(Ci):
                # numpy.correlate(a, v, 'same') with a length-5 kernel centres tap 2 on n
                acc += np.correlate(X[b, :, c], W[o, :, c], mode="same")
            np.testing.assert_allclose(Z[b, :, o], acc, rtol=1e-12, atol=1e-12)


def _torch_net(params, noise, cond, M, L, target):
    items = R.unpack(params, M, L)
    X = torch.tensor(R.net_input(noise, cond).transpose(0, 2, 1))  # [B][C][N]
    ws = []
    for i, (W, b) in enumerate(items):
        Wt = torch.tensor(W.transpose(0, 2, 1).copy(), requires_grad=True)  # [o][c][tap]
        bt = torch.tensor(b.copy(), requires_grad=True)
        ws.append((Wt, bt))
        X = torch.nn.functional.conv1d(X, Wt, bt, padding=2)
        if i < 3:
            X = torch.relu(X)
    B, _, N = X.shape
    z = X.reshape(B, M, L, N).permute(0, 1, 3, 2)  # [B][M][N][L]
    loss = torch.nn.functional.cross_entropy(z.reshape(-1, L), torch.tensor(target.reshape(-1).astype(np.int64)))
    loss.backward()
    g = np.concatenate([np.concatenate([Wt.grad.numpy().transpose(0, 2, 1).reshape(-1), bt.grad.numpy()])
                        for Wt, bt in ws])
    return z.detach().numpy(), float(loss.detach()), g


def test_forward_backward_against_torch_autograd():
    params, noise, cond, B, M, N, L = _small()
    target = I.net_targets(B, M, N, L, 3)
    z, cache = R.forward(params, noise, cond, M, L, rounding=False)
    loss, dz = R.cross_entropy(z, target)
    g = R.backward(cache, dz)
    zt, lt, gt = _torch_net(params, noise, cond, M, L, target)
    np.testing.assert_allclose(z, zt, rtol=1e-12, atol=1e-12)
    assert abs(loss - lt) < 1e-12
    np.testing.assert_allclose(g, gt, rtol=1e-10, atol=1e-13)


def test_gradient_central_differences():
    params, noise, cond, B, M, N, L = _small(seed=5, N=8)
    target = I.net_targets(B, M, N, L, 7)
    p64 = params.astype(np.float64)

    def f(p):
        z, _ = R.forward(p, noise, cond, M, L, rounding=False)
        return R.cross_entropy(z, target)[0]

    z, cache = R.forward(p64, noise, cond, M, L, rounding=False)
    g = R.backward(cache, R.cross_entropy(z, target)[1])
    rng = np.random.default_rng(11)
    for i in rng.choice(p64.size, 24, replace=False):
        e = np.zeros_like(p64)
        e[i] = 1e-6
        fd = (f(p64 + e) - f(p64 - e)) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_cross_entropy_closed_forms():
    rng = np.random.default_rng(2)
    z = rng.standard_normal((2, 3, 5, 8))
    t = rng.integers(0, 8, size=(2, 3, 5))
    loss, dz = R.cross_entropy(z, t)
    np.testing.assert_allclose(dz.sum(axis=-1), 0.0, atol=1e-15)
    # uniform logits: loss = log L
    l0, _ = R.cross_entropy(np.zeros((1, 1, 4, 8)), np.zeros((1, 1, 4), dtype=int))
    assert abs(l0 - np.log(8.0)) < 1e-14


def test_rounded_network_stays_close_to_exact():
    params, noise, cond, B, M, N, L = _small(seed=9, N=64)
    z1, _ = R.forward(params, noise, cond, M, L, rounding=True)
    z0, _ = R.forward(params, noise, cond, M, L, rounding=False)
    rel = np.linalg.norm(z1 - z0) / np.linalg.norm(z0)
    assert 0 < rel < 2e-2  # bfloat16 keeps 8 significant bits

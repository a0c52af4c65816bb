"""The warm-start network's MFMA kernels (through the C ABI) against the FP64
oracle that rounds to bfloat16 at the same places.

Tolerances: the device accumulates in FP32 in another order than the oracle's
FP64, so an intermediate value that sits at a bfloat16 rounding midpoint can
round the other way (one bfloat16 step, 2^-8 relative) and carry that through
the later layers; normwise errors stay below 1e-3 and every element within
1e-2 of the largest magnitude."""
import numpy as np
import pytest

from paper_2604_25728_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def NN():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_25728_amd import native, netnative
    native.load()
    return netnative


def _rel(a, b):
    a, b = np.asarray(a, dtype=np.float64).ravel(), np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _maxrel(a, b):
    a, b = np.asarray(a, dtype=np.float64).ravel(), np.asarray(b, dtype=np.float64).ravel()
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


SHAPES = [(4, 512, 8, 2), (2, 128, 8, 3), (4, 64, 4, 2), (2, 192, 32, 1)]


@pytest.mark.parametrize("M,N,L,B", SHAPES)
def test_forward_and_backward_match_oracle(NN, M, N, L, B):
    from oracle import net_ref as R
    print(f"[gpu] net M={M} N={N} L={L} B={B}", flush=True)
    cond = (L / 8.0, 1.0)
    params = I.net_init(M, L, 1) * 2.0  # larger weights: more active units
    noise = I.net_noise(B, M, N, 2)
    target = I.net_targets(B, M, N, L, 3)
    net = NN.Net(M, N, L, B, cond=cond, params=params)
    z = net.forward(torch.tensor(noise, device="cuda")).cpu().numpy()
    zr, cache = R.forward(params, noise, cond, M, L, rounding=True)
    assert _rel(z, zr) <= 1e-3 and _maxrel(z, zr) <= 1e-2, (_rel(z, zr), _maxrel(z, zr))
    # cross-entropy gradient (the device feeds its own logits; the oracle its own)
    net.backward(target=torch.tensor(target, device="cuda"))
    torch.cuda.synchronize()
    g = net.grad.cpu().numpy()
    loss_ref, dz_ref = R.cross_entropy(zr, target)
    g_ref = R.backward(cache, dz_ref)
    assert abs(net.loss.item() - loss_ref) <= 1e-4 * loss_ref
    off = 0
    for ci, co in I.net_layers(M, L):  # per layer, weights and bias
        n = co * 5 * ci + co
        assert _rel(g[off: off + n], g_ref[off: off + n]) <= 1e-3, (ci, co, _rel(g[off: off + n], g_ref[off: off + n]))
        off += n
    # a given upstream gradient
    gl = np.random.default_rng(4).standard_normal(zr.shape).astype(np.float32)
    net.backward(grad_logits=torch.tensor(gl, device="cuda"))
    torch.cuda.synchronize()
    assert _rel(net.grad.cpu().numpy(), R.backward(cache, gl.astype(np.float64))) <= 1e-3


def test_adam_matches_oracle(NN):
    from oracle import sqngd_ref as SR
    M, N, L, B = 4, 64, 8, 1
    net = NN.Net(M, N, L, B)
    rng = np.random.default_rng(5)
    p0 = net.params.cpu().numpy().astype(np.float64)
    m = np.zeros_like(p0)
    v = np.zeros_like(p0)
    p = p0.copy()
    for t in range(1, 4):
        g = rng.standard_normal(p0.size).astype(np.float32)
        net.grad.copy_(torch.tensor(g))
        net.adam(lr=1e-2)
        p, m, v = SR.adam(p, g.astype(np.float64), m, v, t, 1e-2, 0.9, 0.999, 1e-8)
    torch.cuda.synchronize()
    assert _rel(net.params.cpu().numpy(), p) <= 1e-6


def test_backward_is_deterministic(NN):
    M, N, L, B = 4, 512, 8, 4
    net = NN.Net(M, N, L, B, seed=7)
    noise = torch.tensor(I.net_noise(B, M, N, 8), device="cuda")
    t = torch.tensor(I.net_targets(B, M, N, L, 9), device="cuda")
    net.forward(noise)
    g1 = net.backward(target=t).clone()
    net.forward(noise)
    g2 = net.backward(target=t).clone()
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)


def test_training_overfits_a_small_batch(NN):
    M, N, L, B = 4, 128, 8, 2
    net = NN.Net(M, N, L, B, seed=3)
    noise = torch.tensor(I.net_noise(B, M, N, 10), device="cuda")
    t = torch.tensor(I.net_targets(B, M, N, L, 11), device="cuda")
    first = None
    for i in range(300):
        loss = net.train_step(noise, t, lr=3e-3)
        if i == 0:
            first = loss.item()
    torch.cuda.synchronize()
    last = net.loss.item()
    print(f"overfit: {first:.4f} -> {last:.4f}")
    assert first > 1.9 and last < 0.5 * first

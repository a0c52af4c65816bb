"""The paper's sequence length N = 1200 (FFT length 4096: the throughput pass
spreads one transform over eight waves with three LDS exchanges) against the
FP64 oracle: statistics, AF rows, both gradients, with and without ROI
weights, and two optimiser iterations (whose finalize runs in k_final).
Tolerances as in test_gpu_parity."""
import numpy as np
import pytest

from paper_2604_25728_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def nat():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_25728_amd import native
    native.load()
    return native


def _rel(a, b):
    a, b = np.asarray(a).reshape(-1), np.asarray(b).reshape(-1)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _db(v):
    return 20 * np.log10(v)


@pytest.mark.parametrize("weighted", [False, True])
def test_n1200_evaluation(ref, nat, weighted):
    prob = I.make_problem(2, 1200, 16, 3, nu_min=-0.5, nu_max=0.5, p=16.0, tau_lo=-1100, tau_hi=1150)
    M, N, L = prob["M"], prob["N"], prob["L"]
    print(f"[gpu] N=1200 weighted={weighted}", flush=True)
    z, h = I.logits(M, N, L, 80), I.complex_gaussian(M, N, 81)
    w = I.roi_weights(prob, 82) if weighted else None
    b = nat.Batch([prob])
    if weighted:
        b.set_roi_weights([w])
    zt, ht = b.pack_z([z]), b.pack_w([h])
    stats_f, cube = b.af_forward(zt, ht, nat.WAVE_SOFT, cube=True)
    stats_b = b.new_stats()
    gz, gh, gs = b.af_backward(zt, ht, nat.WAVE_SOFT, want_s=True, stats=stats_b)
    torch.cuda.synchronize()
    s = ref.soft_waveform(z.astype(np.float64), prob["temperature"])
    hr = h.astype(np.complex128)
    pw = dict(prob, roi_w=None if w is None else w.astype(np.float64))
    st_ref, gs_ref, gh_ref = ref.evaluate(s, hr, pw)
    c = b.unpack_cube(cube, 0).cpu().numpy()
    amax = np.abs(c).max()
    for m, l, f in ((0, 0, 0), (0, 1, 2), (1, 0, 1), (1, 1, 2)):
        row = ref.af_row(s, hr, prob["F"], prob["nu_min"], prob["nu_max"], m, l, f)
        assert np.abs(c[m, l, f] - row).max() <= 1e-4 * amax, (m, l, f)
    for st in (nat.decode_stats(stats_f.cpu().numpy())[0], nat.decode_stats(stats_b.cpu().numpy())[0]):
        assert abs(st["loss"] - st_ref["loss"]) <= 1e-4 * st_ref["loss"], (st, st_ref)
        for k in ("psl_auto", "psl_cross"):
            assert abs(_db(st[k]) - _db(st_ref[k])) <= 0.05, (k, st[k], st_ref[k])
        assert abs(st["snrl_db_max"] - st_ref["snrl_db_max"]) <= 0.05
    assert _rel(gs.cpu().numpy(), gs_ref) <= 1e-4
    assert _rel(gh.cpu().numpy(), gh_ref) <= 1e-4
    gz_ref = ref.logit_grad(z.astype(np.float64), prob["temperature"], gs_ref)
    assert _rel(gz.cpu().numpy(), gz_ref) <= 1e-4


def test_n1200_steps(ref, nat):
    from paper_2604_25728_amd import optim
    prob = I.make_problem(2, 1200, 4, 3, p=16.0)
    opt = I.make_opt(total_iters=10, T0=1.0, T1=0.5)
    print("[gpu] N=1200 steps", flush=True)
    run = optim.SQNGD([prob], opt, seeds=[83])
    s0 = run.numpy_state(0)
    run.step(2)
    torch.cuda.synchronize()
    s1 = run.numpy_state(0)
    z, h, state = s0["z"], s0["h"], s0["state"]
    for t in range(2):
        z, h, state, sta, stb = ref.step(prob, opt, z, h, state, t)
    assert s1["t"] == 2
    assert _rel(s1["h"], h) <= 1e-4, _rel(s1["h"], h)
    assert _rel(s1["z"], z) <= 1e-4, _rel(s1["z"], z)
    sa, sb = run.step_stats()
    assert abs(sa[0]["loss"] - sta["loss"]) <= 1e-4 * sta["loss"]
    assert abs(sb[0]["loss"] - stb["loss"]) <= 1e-4 * stb["loss"]

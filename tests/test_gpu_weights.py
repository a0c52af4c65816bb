"""ROI weights w(tau, f) of eq. 8-9 on the GPU (sqngd_set_roi_weights) against
the weighted FP64 oracle: statistics (WAPSL, WCPSL, L_p of w |A| / N) and both
gradients in the throughput and the latency pass, one optimiser step, and the
return to w = 1. Tolerances as in test_gpu_parity."""
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


CASES = {
    "m2n64": (I.config("m2n64")["problem"], 1),
    "ragged": (I.make_problem(3, 100, 5, 7, nu_min=-1.3, nu_max=0.7, p=6.0, tau_lo=-40, tau_hi=30,
                              w_snrl=1.7, temperature=0.6), 1),
    "m4n256_split12": (I.config("m4n256")["problem"], 12),
    "m4n256_throughput": (I.config("m4n256")["problem"], 1),
    "n512_split8": (I.make_problem(2, 512, 4, 5, p=16.0), 8),
    "n1024": (I.make_problem(2, 1024, 4, 3, nu_min=-2.5, nu_max=2.5, p=16.0), 1),
}


@pytest.mark.parametrize("name", list(CASES))
def test_weighted_stats_and_gradients(ref, nat, name):
    prob, sched = CASES[name]
    M, N, L = prob["M"], prob["N"], prob["L"]
    print(f"[gpu] ROI weights {name}", flush=True)
    w = I.roi_weights(prob, 60)
    z, h = I.logits(M, N, L, 61), I.complex_gaussian(M, N, 62)
    b = nat.Batch([dict(prob, schedule=sched)])
    b.set_roi_weights([w])
    zt, ht = b.pack_z([z]), b.pack_w([h])
    stats_f, cube = b.af_forward(zt, ht, nat.WAVE_SOFT, cube=True)
    stats_b = b.new_stats()
    gz, gh, gs = b.af_backward(zt, ht, nat.WAVE_SOFT, want_s=True, stats=stats_b)
    torch.cuda.synchronize()
    s = ref.soft_waveform(z.astype(np.float64), prob["temperature"])
    hr = h.astype(np.complex128)
    pw = dict(prob, roi_w=w.astype(np.float64))
    st_ref, gs_ref, gh_ref = ref.evaluate(s, hr, pw)
    # the cube is the unweighted AF
    cref = ref.af_cube(s, hr, prob["F"], prob["nu_min"], prob["nu_max"])
    c = b.unpack_cube(cube, 0).cpu().numpy()
    assert np.abs(c - cref).max() <= 1e-4 * np.abs(cref).max()
    for st in (nat.decode_stats(stats_f.cpu().numpy())[0], nat.decode_stats(stats_b.cpu().numpy())[0]):
        assert abs(st["loss"] - st_ref["loss"]) <= 1e-4 * st_ref["loss"], (st, st_ref)
        assert abs(st["lp"] - st_ref["lp"]) <= 1e-4 * st_ref["lp"]
        for k in ("psl_auto", "psl_cross"):
            if st_ref[k] > 0:
                assert abs(_db(st[k]) - _db(st_ref[k])) <= 0.05, (k, st[k], st_ref[k])
        assert abs(st["pslr_db"] - st_ref["pslr_db"]) <= 0.05
    assert _rel(gs.cpu().numpy(), gs_ref) <= 1e-4
    assert _rel(gh.cpu().numpy(), gh_ref) <= 1e-4
    gz_ref = ref.logit_grad(z.astype(np.float64), prob["temperature"], gs_ref)
    assert _rel(gz.cpu().numpy(), gz_ref) <= 1e-4
    # the weights matter: the unweighted oracle differs
    st_u = ref.evaluate(s, hr, prob, want_grads=False)[0]
    assert abs(st_u["lp"] - st_ref["lp"]) > 1e-2 * st_ref["lp"]


def test_clearing_weights_restores_the_unweighted_pass(nat):
    prob = I.config("m4n256")["problem"]
    M, N, L = prob["M"], prob["N"], prob["L"]
    print("[gpu] ROI weights cleared", flush=True)
    z, h = I.logits(M, N, L, 63), I.complex_gaussian(M, N, 64)
    b = nat.Batch([prob])
    zt, ht = b.pack_z([z]), b.pack_w([h])
    g0 = b.af_backward(zt, ht, nat.WAVE_SOFT)[0].clone()
    b.set_roi_weights([I.roi_weights(prob, 65)])
    gw = b.af_backward(zt, ht, nat.WAVE_SOFT)[0].clone()
    b.set_roi_weights(None)
    g1 = b.af_backward(zt, ht, nat.WAVE_SOFT)[0].clone()
    torch.cuda.synchronize()
    assert torch.equal(g0, g1)
    assert not torch.equal(g0, gw)


def test_weighted_window_step_matches_oracle(ref, nat):
    """Two outer iterations with the paper's fixed delay window |tau| <= 50 given
    as 0/1 weights, against the oracle's iterations from the same start."""
    from paper_2604_25728_amd import optim
    prob = I.make_problem(2, 128, 4, 9, p=8.0)
    opt = I.make_opt(total_iters=10, T0=1.0, T1=0.5)
    w = I.roi_window_weights(prob, 50)
    print("[gpu] ROI window step", flush=True)
    run = optim.SQNGD([prob], opt, seeds=[66], roi_weights=[w])
    s0 = run.numpy_state(0)
    run.step(2)
    torch.cuda.synchronize()
    s1 = run.numpy_state(0)
    pw = dict(prob, roi_w=w.astype(np.float64))
    z, h, state = s0["z"], s0["h"], s0["state"]
    for t in range(2):
        z, h, state, sta, stb = ref.step(pw, opt, z, h, state, t)
    assert _rel(s1["h"], h) <= 1e-4, _rel(s1["h"], h)
    assert _rel(s1["z"], z) <= 1e-4, _rel(s1["z"], z)
    sa, sb = run.step_stats()
    assert abs(sb[0]["loss"] - stb["loss"]) <= 1e-4 * stb["loss"]
    # the window equals the delay ROI tau_lo = -50, tau_hi = 50 without weights
    pn = dict(prob, tau_lo=-50, tau_hi=50)
    z2, h2, st2 = s0["z"], s0["h"], s0["state"]
    for t in range(2):
        z2, h2, st2, _, _ = ref.step(pn, opt, z2, h2, st2, t)
    assert _rel(z2, z) <= 1e-10 and _rel(h2, h) <= 1e-10


def test_subset_keeps_weights(nat):
    from paper_2604_25728_amd import optim
    c = I.config("m2n64")
    print("[gpu] ROI weights subset", flush=True)
    ws = [I.roi_weights(c["problem"], 70 + i) for i in range(3)]
    a = optim.SQNGD([c["problem"]] * 3, c["opt"], seeds=[5, 6, 7], schedule=nat.SCHED_THROUGHPUT, roi_weights=ws)
    a.run(4, use_graph=False)
    sub = a.subset([2])
    a.run(4, use_graph=False)
    sub.run(4, use_graph=False)
    torch.cuda.synchronize()
    assert torch.equal(sub.batch.unpack_z(sub.z, 0), a.batch.unpack_z(a.z, 2))
    assert torch.equal(sub.batch.unpack_roi(0), a.batch.unpack_roi(2))

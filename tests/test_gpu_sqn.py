"""The paper's transmit parameterisation on the GPU (include/sqngd_sqn.h)
against its FP64 oracle: the ResNet forward and backward, the copied tanh
staircase and its gradients, the hard quantiser (bit-exact away from the
thresholds), Adam, the threshold sort, the filter projection, and two outer
iterations of Algorithm 1 with this transmit side.

Tolerances: the network and the staircase run in FP32 against FP64; outputs
within 1e-5 relative normwise, soft-waveform phases within 1e-4 rad,
gradients within 1e-4 (the staircase sums K tanh terms); the iteration as in
test_gpu_optim (1e-4), and at the paper's staircase (c = 300, r_n = 100) the
parameter updates themselves within 1e-3 of the oracle's."""
import numpy as np
import pytest

from paper_2604_25728_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def SN():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_25728_amd import native, sqnnative
    native.load()
    return sqnnative


@pytest.fixture(scope="module")
def S():
    from oracle import sqn_ref
    return sqn_ref


def _rel(a, b):
    a, b = np.asarray(a).reshape(-1), np.asarray(b).reshape(-1)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _t(a, dtype=torch.float32):
    return torch.as_tensor(np.asarray(a)).to(dtype).cuda().contiguous()


@pytest.mark.parametrize("M,N,B,copies,c", [(2, 64, 4, 3, 30.0), (3, 100, 16, 10, 100.0), (2, 512, 4, 100, 300.0)])
def test_network_and_staircase(SN, S, M, N, B, copies, c):
    D = M * N
    print(f"[gpu] sqn M={M} N={N} B={B} copies={copies}", flush=True)
    q = SN.SQN(M, N, B, copies, c)
    theta = I.sqn_init(D, 20)
    y0 = I.sqn_input(M, N, B, 21)
    rho = I.sqn_thresholds(B, copies) + np.random.default_rng(22).normal(0, 1e-4, B * copies).astype(np.float32)
    rho = np.sort(rho).astype(np.float32)
    th, y, r = _t(theta), _t(y0), _t(rho)
    z = q.forward(th, y)
    s = q.soft(z, r)
    idx, x = q.hard(z, r)
    torch.cuda.synchronize()
    zr, cache = S.forward(theta.astype(np.float64), y0.astype(np.float64))
    assert _rel(z.cpu().numpy(), zr) <= 1e-5
    # the staircase on the GPU's own z (the FP32 network's rounding stays out of this check)
    zg = z.cpu().numpy().astype(np.float64)
    y1 = S.soft_quantise(zg, rho.astype(np.float64), B, c)
    # (the phase is formed from the threshold count mod B plus the fractional
    # terms, so FP32 keeps ~1e-6 rad whatever the copy count)
    assert np.abs(np.angle(s.cpu().numpy() * np.conj(np.exp(2j * np.pi * y1)))).max() <= 1e-4
    k_ref = S.hard_levels(zg, rho.astype(np.float64)) % B
    far = np.min(np.abs(zg[:, None] - rho[None, :].astype(np.float64)), axis=1) > 1e-6
    assert np.array_equal(idx.cpu().numpy()[far], k_ref[far])
    assert np.allclose(x.cpu().numpy(), np.exp(2j * np.pi * idx.cpu().numpy() / B), atol=1e-6)
    # backward from a given waveform gradient
    gs = (np.random.default_rng(23).standard_normal(D) + 1j * np.random.default_rng(24).standard_normal(D))
    gt, gr = q.backward(th, y, z, r, s, _t(gs, torch.complex64))
    torch.cuda.synchronize()
    sg = s.cpu().numpy().astype(np.complex128)
    dy = S.waveform_chain(gs.astype(np.complex64).astype(np.complex128), sg)
    dz, drho = S.soft_quantise_grad(zg, rho.astype(np.float64), B, c, dy)
    _, cache_g = S.forward(theta.astype(np.float64), y0.astype(np.float64))
    cache_g["z"] = zg
    dth = S.backward(cache_g, dz)
    assert _rel(gr.cpu().numpy(), drho) <= 1e-4, _rel(gr.cpu().numpy(), drho)
    assert _rel(gt.cpu().numpy(), dth) <= 1e-4, _rel(gt.cpu().numpy(), dth)
    # with a filter gradient (matched filtering): the two add before the chain
    gh = np.random.default_rng(25).standard_normal(D) - 0.5j * np.random.default_rng(26).standard_normal(D)
    gt2, gr2 = q.backward(th, y, z, r, s, _t(gs, torch.complex64), _t(gh, torch.complex64))
    torch.cuda.synchronize()
    g2 = gs.astype(np.complex64).astype(np.complex128) + gh.astype(np.complex64).astype(np.complex128)
    dz2, drho2 = S.soft_quantise_grad(zg, rho.astype(np.float64), B, c, S.waveform_chain(g2, sg))
    assert _rel(gr2.cpu().numpy(), drho2) <= 1e-4, _rel(gr2.cpu().numpy(), drho2)
    assert _rel(gt2.cpu().numpy(), S.backward(cache_g, dz2)) <= 1e-4
    # backward + Adam on theta in one call equals backward then Adam, bit for bit
    m0 = torch.zeros_like(th)
    v0 = torch.zeros_like(th)
    th_a, m_a, v_a = th.clone(), m0.clone(), v0.clone()
    th_b, m_b, v_b = th.clone(), m0.clone(), v0.clone()
    q.forward(th, y)  # the activations of theta in the workspace
    gt3, gr3 = q.backward(th, y, z, r, s, _t(gs, torch.complex64))
    SN.adam(th_a, gt3, m_a, v_a, 1, 1e-3, 0.9, 0.999, 1e-8)
    gr4 = q.backward_adam(th_b, y, z, r, s, _t(gs, torch.complex64), m_b, v_b, 1, 1e-3, 0.9, 0.999, 1e-8)
    torch.cuda.synchronize()
    assert torch.equal(th_a, th_b) and torch.equal(m_a, m_b) and torch.equal(v_a, v_b)
    assert torch.equal(gr3, gr4) and not torch.equal(th_b, th)


def test_adam_sort_project(SN, S):
    from oracle import sqngd_ref as R
    rng = np.random.default_rng(30)
    p0, g = rng.standard_normal(1000).astype(np.float32), rng.standard_normal(1000).astype(np.float32)
    p, m, v = _t(p0), torch.zeros(1000, device="cuda"), torch.zeros(1000, device="cuda")
    pr, mr, vr = p0.astype(np.float64), np.zeros(1000), np.zeros(1000)
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    for t in (1, 2, 3):
        SN.adam(p, _t(g), m, v, 1, 1e-2, 0.9, 0.999, 1e-8, step=cnt, step_mul=1)  # t from the device counter
        SN.lib().sqngd_sqn_count(SN._ptr(cnt), SN._stream())
        pr, mr, vr = R.adam(pr, g.astype(np.float64), mr, vr, t, 1e-2, 0.9, 0.999, 1e-8)
    q = SN.SQN(2, 8, 4, 700, 30.0)   # K = 2800 thresholds (padded to 4096 in the sort)
    rho = rng.random(2800).astype(np.float32)
    r = _t(rho)
    q.sort(r)
    # rank path (K <= 1024): ties, signed zeros and infinities
    q2 = SN.SQN(2, 8, 4, 100, 30.0)   # K = 400
    rho2 = np.round(rng.standard_normal(400) * 4).astype(np.float32)
    rho2[:3] = [np.inf, -np.inf, -0.0]
    r2 = _t(rho2)
    q2.sort(r2)
    q3 = SN.SQN(2, 8, 4, 256, 30.0)   # K = 1024, the rank path's largest
    rho3 = rng.random(1024).astype(np.float32)
    r3 = _t(rho3)
    q3.sort(r3)
    # already ordered (the comparison pass skips the network), with ties
    rho4 = np.sort(np.round(rng.random(400) * 50).astype(np.float32))
    r4 = _t(rho4)
    q2.sort(r4)
    h = (rng.standard_normal((2, 8)) + 1j * rng.standard_normal((2, 8))).astype(np.complex64)
    ht = _t(h, torch.complex64).reshape(-1)
    q.project(ht)
    torch.cuda.synchronize()
    assert _rel(p.cpu().numpy(), pr) <= 1e-6
    assert np.array_equal(r.cpu().numpy(), np.sort(rho))
    assert np.array_equal(r2.cpu().numpy(), np.sort(rho2))
    assert np.array_equal(r3.cpu().numpy(), np.sort(rho3))
    assert np.array_equal(r4.cpu().numpy(), rho4)
    assert _rel(ht.cpu().numpy().reshape(2, 8), R.project(h.astype(np.complex128))) <= 1e-6


def test_fused_adam_entry_points_match_separate_calls(SN):
    """sqngd_sqn_adam_project and sqngd_sqn_adam_sort equal sqngd_sqn_adam
    followed by sqngd_sqn_project / sqngd_sqn_sort, bit for bit (three
    stacked designs, step count from a device counter)."""
    rng = np.random.default_rng(31)
    print("[gpu] sqn fused adam", flush=True)
    cnt = torch.tensor([2], dtype=torch.int32, device="cuda")
    rows, N, K, R = 6, 100, 400, 3
    h0 = (rng.standard_normal(rows * N) + 1j * rng.standard_normal(rows * N)).astype(np.complex64)
    g = (rng.standard_normal(rows * N) + 1j * rng.standard_normal(rows * N)).astype(np.complex64)
    m0 = rng.standard_normal(2 * rows * N).astype(np.float32) * 0.1
    v0 = rng.random(2 * rows * N).astype(np.float32) * 0.1
    ha, ma, va = _t(h0, torch.complex64), _t(m0), _t(v0)
    hb, mb, vb = ha.clone(), ma.clone(), va.clone()
    gt = _t(g, torch.complex64)
    SN.adam(torch.view_as_real(ha).reshape(-1), torch.view_as_real(gt).reshape(-1), ma, va, 3, 5e-2, 0.9, 0.999,
            1e-8, step=cnt, step_mul=10)
    SN.lib().sqngd_sqn_project(rows, N, SN._ptr(ha), SN._stream())
    SN.adam_project(hb, gt, mb, vb, rows, N, 3, 5e-2, 0.9, 0.999, 1e-8, step=cnt, step_mul=10)
    rho0 = np.sort(rng.random((R, K)).astype(np.float32), axis=1).reshape(-1)
    gr = _t(rng.standard_normal(R * K).astype(np.float32))
    ra, rb = _t(rho0), _t(rho0)
    mra, vra = torch.zeros(R * K, device="cuda"), torch.zeros(R * K, device="cuda")
    mrb, vrb = mra.clone(), vra.clone()
    SN.adam(ra, gr, mra, vra, 1, 1e-2, 0.9, 0.999, 1e-8, step=cnt, step_mul=10)
    SN.lib().sqngd_sqn_sort(SN._ptr(ra), K, R, SN._stream())
    SN.adam_sort(rb, gr, mrb, vrb, K, R, 1, 1e-2, 0.9, 0.999, 1e-8, step=cnt, step_mul=10)
    torch.cuda.synchronize()
    assert torch.equal(ha, hb) and torch.equal(ma, mb) and torch.equal(va, vb)
    assert torch.equal(ra, rb) and torch.equal(mra, mrb) and torch.equal(vra, vrb)
    assert np.all(np.diff(rb.cpu().numpy().reshape(R, K), axis=1) >= 0)
    assert not torch.equal(rb, _t(rho0))


def test_two_iterations_match_oracle(SN, S):
    """Two outer iterations (n_h = n_x = 1) from the same state: filters,
    network parameters and thresholds against the oracle's. A gentle
    staircase (c = 4) keeps every threshold's gradient far above FP32
    resolution: Adam's step is about lr times the sign of a gradient, so a
    threshold whose gradient underflows in FP32 (tanh saturates) would move
    by lr in the oracle and not at all on the GPU."""
    prob = I.make_problem(2, 64, 4, 5, p=8.0)
    opt = I.make_opt(lr_z=1e-3, lr_h=1e-2)
    copies, c = 3, 4.0
    print("[gpu] sqn iterations", flush=True)
    d = SN.SQNDesign(prob, opt, copies, c, seed=40)
    theta0 = d.theta.cpu().numpy().astype(np.float64)
    rho0 = d.rho.cpu().numpy().astype(np.float64)
    y0 = d.y0.cpu().numpy().astype(np.float64)
    h0 = d.h.cpu().numpy().reshape(2, 64).astype(np.complex128)
    for _ in range(2):
        d.iteration()
    torch.cuda.synchronize()
    th, rho, h, st = theta0, rho0, h0, S.new_state(2 * 64, 4 * copies, 2, 64)
    for t in range(2):
        th, rho, h, st, sa, sb = S.iteration(prob, opt, {"c": c, "copies": copies}, th, rho, h, y0, st, t)
    assert _rel(d.h.cpu().numpy().reshape(2, 64), h) <= 1e-4, _rel(d.h.cpu().numpy().reshape(2, 64), h)
    assert _rel(d.theta.cpu().numpy(), th) <= 1e-4, _rel(d.theta.cpu().numpy(), th)
    assert _rel(d.rho.cpu().numpy(), rho) <= 1e-4
    assert np.all(np.diff(d.rho.cpu().numpy()) >= 0)
    from paper_2604_25728_amd import native as nat
    stb = nat.decode_stats(d.stats_b.cpu().numpy())[0]
    assert abs(stb["loss"] - sb["loss"]) <= 1e-4 * sb["loss"]


def test_initialisation_follows_algorithm_1(SN, S):
    """Algorithm 1's start: y0 holds discrete normalised phases b / B, and the
    filters are the projected matched filter of X0 = exp(j 2 pi Y0)."""
    prob = I.make_problem(2, 64, 4, 5, p=8.0)
    d = SN.SQNDesign(prob, I.make_opt(), 3, 30.0, seed=[70, 71])
    y0 = d.y0.cpu().numpy().astype(np.float64).reshape(2, 2 * 64)
    assert np.array_equal(y0 * 4, np.round(y0 * 4)) and y0.min() >= 0 and y0.max() <= 0.75
    h = d.h.cpu().numpy().reshape(2, 2, 64)
    for r in range(2):
        want = S.initial_filters(y0[r], 2, 64)
        assert np.abs(h[r] - want).max() <= 1e-6
        assert np.allclose(np.abs(np.sum(np.conj(h[r]) * np.exp(2j * np.pi * y0[r].reshape(2, 64)), axis=1)), 64)


def test_paper_staircase_iterations_match_oracle(SN, S):
    """Two outer iterations at the paper's transmit settings (r_n = 100 copies,
    c = 300, B = 4, M = 2, N = 512, eps = 0.1, |tau| <= 50 as ROI weights,
    N_h = N_x = 2) against the oracle from the same state. At c = 300 most
    thresholds sit where tanh rounds to +-1 in FP32: their gradients come
    from the cancellation-free slope 4e / (1 + e)^2, so they move on the GPU
    as in the oracle. Compared: the updates of theta, rho and h (normwise,
    1e-3: a handful of parameters whose gradient is within FP32 rounding of
    zero may take Adam's step with the other sign) and the step-B loss."""
    prob = I.make_problem(2, 512, 4, 9, p=16.0, w_psl=0.1, w_snrl=0.9)
    opt = I.make_opt(lr_z=1e-5, lr_h=5e-2, n_h=2, n_x=2)
    copies, c = 100, 300.0
    print("[gpu] sqn iterations at c=300 r_n=100", flush=True)
    d = SN.SQNDesign(prob, opt, copies, c, seed=42)
    w = I.roi_window_weights(prob, 50)
    d.batch.set_roi_weights([w])
    theta0 = d.theta.cpu().numpy().astype(np.float64)
    rho0 = d.rho.cpu().numpy().astype(np.float64)
    y0 = d.y0.cpu().numpy().astype(np.float64)
    h0 = d.h.cpu().numpy().reshape(2, 512).astype(np.complex128)
    for _ in range(2):
        d.iteration()
    torch.cuda.synchronize()
    pw = dict(prob, roi_w=w.astype(np.float64))
    th, rho, h, st = theta0, rho0, h0, S.new_state(2 * 512, 4 * copies, 2, 512)
    for t in range(2):
        th, rho, h, st, sa, sb = S.iteration(pw, opt, {"c": c, "copies": copies}, th, rho, h, y0, st, t)
    d_th = _rel(d.theta.cpu().numpy() - theta0, th - theta0)
    d_rho = _rel(d.rho.cpu().numpy() - rho0, rho - rho0)
    d_h = _rel(d.h.cpu().numpy().reshape(2, 512) - h0, h - h0)
    print(f"update errors: theta {d_th:.2e} rho {d_rho:.2e} h {d_h:.2e}", flush=True)
    # thresholds at least 9 / c from every chip (tanh rounds to +-1 in FP32
    # there) that still take a sizeable step in the oracle move the same on
    # the GPU
    z0, _ = S.forward(theta0, y0)
    far = np.min(np.abs(z0[:, None] - rho0[None, :]), axis=0) * c > 9.0
    step_ref, step_gpu = rho - rho0, d.rho.cpu().numpy() - rho0
    sel = far & (np.abs(step_ref) > 0.1 * opt["lr_z"])
    print(f"{far.sum()} thresholds in the saturated regime, {sel.sum()} of them moving", flush=True)
    assert sel.sum() > 0
    close = np.abs(step_gpu - step_ref)[sel] <= 0.1 * np.abs(step_ref)[sel]
    assert close.mean() >= 0.99, close.mean()
    assert d_th <= 1e-3 and d_rho <= 1e-3 and d_h <= 1e-3
    assert np.all(np.diff(d.rho.cpu().numpy()) >= 0)
    from paper_2604_25728_amd import native as nat
    stb = nat.decode_stats(d.stats_b.cpu().numpy())[0]
    assert abs(stb["loss"] - sb["loss"]) <= 1e-4 * sb["loss"]


def test_matched_filter_mode_matches_oracle(SN, S):
    """The AF extension of SQN (no filter optimisation, the filters are the
    waveform): two outer iterations with n_x = 2 against the oracle's matched
    mode; the filter gradient of the same evaluation adds to the waveform's
    inside sqngd_sqn_backward. The hard evaluation uses h = x."""
    prob = I.make_problem(2, 64, 4, 5, p=8.0, snrl_target_db=0.0)
    opt = I.make_opt(lr_z=1e-3, lr_h=1e-2, n_h=3, n_x=2)
    copies, c = 3, 4.0
    print("[gpu] sqn matched-filter iterations", flush=True)
    d = SN.SQNDesign(prob, opt, copies, c, seed=41, matched=True)
    theta0 = d.theta.cpu().numpy().astype(np.float64)
    rho0 = d.rho.cpu().numpy().astype(np.float64)
    y0 = d.y0.cpu().numpy().astype(np.float64)
    h0 = d.h.cpu().numpy().reshape(2, 64).astype(np.complex128)
    for _ in range(2):
        d.iteration()
    torch.cuda.synchronize()
    th, rho, h, st = theta0, rho0, h0, S.new_state(2 * 64, 4 * copies, 2, 64)
    for t in range(2):
        th, rho, h, st, sa, sb = S.iteration(prob, opt, {"c": c, "copies": copies}, th, rho, h, y0, st, t,
                                             matched=True)
    assert sa is None
    assert _rel(d.theta.cpu().numpy(), th) <= 1e-4, _rel(d.theta.cpu().numpy(), th)
    assert _rel(d.rho.cpu().numpy(), rho) <= 1e-4
    from paper_2604_25728_amd import native as nat
    stb = nat.decode_stats(d.stats_b.cpu().numpy())[0]
    assert abs(stb["loss"] - sb["loss"]) <= 1e-4 * sb["loss"]
    # hard evaluation with matched filtering: SNRL 0 dB (h = x)
    hs = d.hard_stats()
    assert abs(hs["snrl_db_max"]) <= 1e-4
    # the oracle evaluates the GPU's own hard levels (a level at a threshold
    # could flip between FP32 and FP64 parameters)
    x = np.exp(2j * np.pi * d.hard_indices() / 4)
    from oracle import sqngd_ref as R
    ref_st = R.evaluate(x, x, prob, want_grads=False)[0]
    assert abs(hs["psl_auto"] - ref_st["psl_auto"]) <= 1e-4 * ref_st["psl_auto"]


@pytest.mark.parametrize("matched", [False, True])
def test_stacked_designs_match_oracle(SN, S, matched):
    """Three random restarts of one problem stacked (one AF batch of three
    problems, the network with one workgroup per design): two outer
    iterations of each design against the oracle run on its own."""
    prob = I.make_problem(2, 64, 4, 5, p=8.0, snrl_target_db=0.0 if matched else 0.5)
    opt = I.make_opt(lr_z=1e-3, lr_h=1e-2, n_h=1, n_x=1)
    copies, c, seeds = 3, 4.0, [60, 61, 62]
    print(f"[gpu] sqn stacked designs matched={matched}", flush=True)
    d = SN.SQNDesign(prob, opt, copies, c, seed=seeds, matched=matched)
    P, K, D = d.sqn.count, 4 * copies, 2 * 64
    theta0 = d.theta.cpu().numpy().astype(np.float64).reshape(3, P)
    rho0 = d.rho.cpu().numpy().astype(np.float64).reshape(3, K)
    y0 = d.y0.cpu().numpy().astype(np.float64).reshape(3, D)
    h0 = d.h.cpu().numpy().reshape(3, 2, 64).astype(np.complex128)
    for _ in range(2):
        d.iteration()
    torch.cuda.synchronize()
    th_g = d.theta.cpu().numpy().reshape(3, P)
    rho_g = d.rho.cpu().numpy().reshape(3, K)
    h_g = d.h.cpu().numpy().reshape(3, 2, 64)
    from paper_2604_25728_amd import native as nat
    stb = nat.decode_stats(d.stats_b.cpu().numpy())
    for r in range(3):
        th, rho, h, st = theta0[r], rho0[r], h0[r], S.new_state(D, K, 2, 64)
        for t in range(2):
            th, rho, h, st, sa, sb = S.iteration(prob, opt, {"c": c, "copies": copies}, th, rho, h, y0[r], st, t,
                                                 matched=matched)
        assert _rel(th_g[r], th) <= 1e-4, (r, _rel(th_g[r], th))
        assert _rel(rho_g[r], rho) <= 1e-4, r
        assert np.all(np.diff(rho_g[r]) >= 0)
        if not matched:
            assert _rel(h_g[r], h) <= 1e-4, (r, _rel(h_g[r], h))
        assert abs(stb[r]["loss"] - sb["loss"]) <= 1e-4 * sb["loss"], r
    # the designs differ (own seeds)
    assert not np.allclose(th_g[0], th_g[1])
    assert d.hard_indices().shape == (3, 2, 64) and len(d.hard_stats()) == 3


def test_graph_replay_matches_eager(SN):
    """Replays of a captured outer iteration (step counts from the device
    counter) equal eager iterations, with eager work between the replays."""
    prob = I.make_problem(2, 64, 4, 5, p=8.0)
    opt = I.make_opt(lr_z=1e-3, lr_h=1e-2)
    print("[gpu] sqn graph replay", flush=True)
    a = SN.SQNDesign(prob, opt, 3, 30.0, seed=50)
    b = SN.SQNDesign(prob, opt, 3, 30.0, seed=50)
    a.capture()
    for i in range(3):
        a.graph.replay()
        b.iteration()
        torch.cuda.synchronize()
        _ = (a.theta * 2).sum().item()
        assert torch.equal(a.theta, b.theta) and torch.equal(a.h, b.h) and torch.equal(a.rho, b.rho), i
    assert a.t == b.t == 3

"""The alternating iteration on the GPU against the oracle, HIP-graph replays,
finite differences of the FP32 loss, autograd, non-finite handling and
checkpoint / resume."""
import numpy as np
import pytest

from paper_2604_25728_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_25728_amd import autograd, native, optim
    native.load()
    return native, optim, autograd


def _rel(a, b):
    a, b = np.asarray(a).reshape(-1), np.asarray(b).reshape(-1)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("cfg,warm", [("m2n64", 3), ("m4n256", 2)])
def test_step_teacher_forced(ref, mods, cfg, warm):
    """From the GPU state at iteration t, one oracle iteration matches the GPU's."""
    nat, optim, _ = mods
    c = I.config(cfg)
    prob, opt = c["problem"], c["opt"]
    print(f"[gpu] teacher-forced step {cfg}", flush=True)
    run = optim.SQNGD([prob], opt, seeds=[0])
    for _ in range(warm):
        run.step()
    torch.cuda.synchronize()
    s0 = run.numpy_state(0)
    run.step()
    torch.cuda.synchronize()
    s1 = run.numpy_state(0)
    sa, sb = run.step_stats()
    z, h, state, sta, stb = ref.step(prob, opt, s0["z"], s0["h"], s0["state"], s0["t"])
    assert s1["t"] == s0["t"] + 1
    assert _rel(s1["h"], h) <= 1e-4
    assert _rel(s1["z"], z) <= 1e-4
    assert _rel(s1["state"]["vz"], state["vz"]) <= 1e-3
    assert abs(sa[0]["loss"] - sta["loss"]) <= 1e-4 * sta["loss"]
    assert abs(sb[0]["loss"] - stb["loss"]) <= 1e-4 * stb["loss"]
    assert abs(sa[0]["pslr_db"] - sta["pslr_db"]) <= 0.05
    np.testing.assert_allclose((np.abs(s1["h"]) ** 2).sum(axis=1), prob["N"], rtol=1e-5)


def test_c1_run_matches_oracle_where_margins_are_clear(ref, mods):
    """The full 200-iteration M=2 N=64 design: final hard indices equal the oracle's
    on every chip whose oracle top-2 logit margin exceeds 1e-3 (the rest is
    reported); the final hard PSLR agrees within 0.05 dB."""
    nat, optim, _ = mods
    c = I.config("m2n64")
    prob, opt = c["problem"], c["opt"]
    print("[gpu] M=2 N=64 full run", flush=True)
    run = optim.SQNGD([prob], opt, seeds=[0])
    run.run(opt["total_iters"], use_graph=True)
    torch.cuda.synchronize()
    z0 = I.logits(prob["M"], prob["N"], prob["L"], 0).astype(np.float64)
    z, h = z0, ref.matched_init(z0)
    state = ref.new_state(prob["M"], prob["N"], prob["L"])
    for t in range(opt["total_iters"]):
        z, h, state, _, _ = ref.step(prob, opt, z, h, state, t)
    srt = np.sort(z, axis=-1)
    clear = (srt[..., -1] - srt[..., -2]) > 1e-3
    got = run.hard_indices()[0]
    want = ref.hard_indices(z)
    agree = (got == want)[clear].mean()
    print(f"M=2 N=64 final: {clear.mean():.3f} of chips clear, agreement {agree:.4f}, "
          f"unclear chips agreeing {(got == want)[~clear].mean() if (~clear).any() else 1.0:.3f}")
    assert np.array_equal(got[clear], want[clear]), np.argwhere((got != want) & clear)
    st_gpu = run.hard_stats()[0]
    st_ref = ref.evaluate(ref.hard_waveform(z), h, prob, False)[0]
    print("final PSLR gpu", st_gpu["pslr_db"], "oracle", st_ref["pslr_db"])
    assert abs(st_gpu["pslr_db"] - st_ref["pslr_db"]) <= 0.05
    st0 = ref.evaluate(ref.hard_waveform(z0), ref.matched_init(z0), prob, False)[0]
    assert st_gpu["loss"] < st0["loss"]


def test_graph_replay_matches_eager(mods):
    nat, optim, _ = mods
    c = I.config("m4n256")
    print("[gpu] graph replay vs eager", flush=True)
    a = optim.SQNGD([c["problem"]], c["opt"], seeds=[1])
    b = optim.SQNGD([c["problem"]], c["opt"], seeds=[1])
    a.capture()
    for i in range(4):
        a.replay()
        b.step()
        torch.cuda.synchronize()
        _ = (a.z * 2).sum().item()  # eager work between replays
        assert torch.equal(a.z, b.z) and torch.equal(a.h, b.h), i
        assert torch.equal(a.counter, b.counter)
    assert a.t == 4


def test_checkpoint_resume_bitwise(mods, tmp_path):
    nat, optim, _ = mods
    c = I.config("m2n64")
    print("[gpu] checkpoint resume", flush=True)
    a = optim.SQNGD([c["problem"]], c["opt"], seeds=[2])
    a.run(5, use_graph=False)
    path = tmp_path / "ck.pt"
    torch.save(a.state_dict(), path)
    a.run(5, use_graph=False)
    b = optim.SQNGD([c["problem"]], c["opt"], seeds=[99])
    b.load_state_dict(torch.load(path, weights_only=True))
    b.run(5, use_graph=False)
    torch.cuda.synchronize()
    assert torch.equal(a.z, b.z) and torch.equal(a.h, b.h) and a.t == b.t == 10


def test_nonfinite_skips_update(mods):
    nat, optim, _ = mods
    c = I.config("m2n64")
    print("[gpu] non-finite", flush=True)
    run = optim.SQNGD([c["problem"]], c["opt"], seeds=[3])
    run.z[5] = float("nan")   # chip (0, 1): its soft waveform, hence the step-B loss, is NaN
    z_before = run.z.clone()
    run.step()
    torch.cuda.synchronize()
    sa, sb = run.step_stats()
    assert sb[0]["nonfinite"] == 1
    assert sa[0]["nonfinite"] == 0      # the hard waveform ignores the NaN logit
    same = torch.equal(torch.nan_to_num(run.z, nan=7.0), torch.nan_to_num(z_before, nan=7.0))
    assert same                          # logits were not updated
    assert torch.isfinite(run.h).all()


def test_finite_differences_c2(mods):
    """Central differences (step 1e-3) of the FP32 loss on 32 random coordinates."""
    nat, _, _ = mods
    prob = I.config("m4n256")["problem"]
    M, N, L = prob["M"], prob["N"], prob["L"]
    print("[gpu] finite differences M=4 N=256", flush=True)
    b = nat.Batch([prob])
    z = b.pack_z([I.logits(M, N, L, 4)])
    h = b.pack_w([I.complex_gaussian(M, N, 5) * 0.9 + I.unimodular(M, N, 6)])
    gz, gh, _ = b.af_backward(z, h, nat.WAVE_SOFT)
    torch.cuda.synchronize()
    gz, gh = gz.cpu().numpy(), gh.cpu().numpy()
    rng = np.random.default_rng(7)

    def loss(zz, hh):
        st = b.af_forward(zz, hh, nat.WAVE_SOFT)
        return float(st.view(torch.float32)[0, 0].item())

    step = 1e-3
    gmax_z, gmax_h = np.abs(gz).max(), np.abs(gh).max()
    for k in range(32):
        if k % 2 == 0:
            i = int(rng.integers(gz.size))
            zp, zm = z.clone(), z.clone()
            zp[i] += step
            zm[i] -= step
            fd = (loss(zp, h) - loss(zm, h)) / (2 * step)
            an, floor = gz[i], 1e-4 * gmax_z
        else:
            i = int(rng.integers(gh.size))
            part = complex(1, 0) if k % 4 == 1 else complex(0, 1)
            hp, hm = h.clone(), h.clone()
            hp[i] += step * part
            hm[i] -= step * part
            fd = (loss(z, hp) - loss(z, hm)) / (2 * step)
            an, floor = (gh[i].real if part.real else gh[i].imag), 1e-4 * gmax_h
        tol = max(1e-3 * abs(an), floor, 2e-7 / step)
        assert abs(fd - an) <= tol, (k, i, fd, an, tol)


def test_autograd_function(ref, mods):
    nat, _, ag = mods
    prob = I.make_problem(2, 48, 4, 5, p=8.0, nu_min=-0.7, nu_max=0.7)
    print("[gpu] autograd", flush=True)
    b = nat.Batch([prob])
    z0 = I.logits(2, 48, 4, 8)
    h0 = I.complex_gaussian(2, 48, 9)
    z = b.pack_z([z0]).requires_grad_(True)
    h = b.pack_w([h0]).requires_grad_(True)
    loss = ag.af_loss(z, h, b, nat.WAVE_SOFT)
    (3.0 * loss.sum()).backward()
    s = ref.soft_waveform(z0.astype(np.float64), 1.0)
    st, gs, gh = ref.evaluate(s, h0.astype(np.complex128), prob)
    gz = ref.logit_grad(z0.astype(np.float64), 1.0, gs)
    assert abs(loss.item() - st["loss"]) <= 1e-4 * st["loss"]
    assert _rel(z.grad.cpu().numpy(), 3.0 * gz) <= 1e-4
    assert _rel(h.grad.cpu().numpy(), 3.0 * gh) <= 1e-4
    # given waveform: gradient with respect to s itself
    sg = b.pack_w([I.unimodular(2, 48, 10)]).requires_grad_(True)
    h2 = h.detach().clone().requires_grad_(True)
    l2 = ag.af_loss(None, h2, b, nat.WAVE_GIVEN, sg)
    l2.sum().backward()
    st2, gs2, gh2 = ref.evaluate(sg.detach().cpu().numpy().astype(np.complex128).reshape(2, 48),
                                 h0.astype(np.complex128), prob)
    assert _rel(sg.grad.cpu().numpy(), gs2) <= 1e-4
    assert _rel(h2.grad.cpu().numpy(), gh2) <= 1e-4


@pytest.mark.parametrize("n_h,n_x", [(1, 1), (2, 2), (0, 1), (1, 0)])
def test_chained_run_matches_oracle(ref, mods, n_h, n_x):
    """sqngd_run over several iterations (updates prepare the next evaluation
    inside the finalize kernel) against the oracle's iterations from the same
    start, for every combination of inner-step counts the chaining handles."""
    nat, optim, _ = mods
    prob = I.config("m2n64")["problem"]
    opt = I.make_opt(n_h=n_h, n_x=n_x, total_iters=20, T0=1.0, T1=0.3)
    print(f"[gpu] chained run n_h={n_h} n_x={n_x}", flush=True)
    run = optim.SQNGD([prob], opt, seeds=[11])
    s0 = run.numpy_state(0)
    iters = 3
    run.step(iters)
    torch.cuda.synchronize()
    s1 = run.numpy_state(0)
    z, h, state = s0["z"], s0["h"], s0["state"]
    for t in range(iters):
        z, h, state, sta, stb = ref.step(prob, opt, z, h, state, t)
    assert s1["t"] == iters
    assert _rel(s1["h"], h) <= 1e-4, _rel(s1["h"], h)
    assert _rel(s1["z"], z) <= 1e-4, _rel(s1["z"], z)
    sa, sb = run.step_stats()
    if n_h:
        assert abs(sa[0]["loss"] - sta["loss"]) <= 1e-4 * sta["loss"]
    if n_x:
        assert abs(sb[0]["loss"] - stb["loss"]) <= 1e-4 * stb["loss"]


def test_chained_graph_matches_eager_run(mods):
    nat, optim, _ = mods
    c = I.config("m4n256")
    print("[gpu] chained graph vs eager run", flush=True)
    a = optim.SQNGD([c["problem"]], c["opt"], seeds=[3])
    b = optim.SQNGD([c["problem"]], c["opt"], seeds=[3])
    a.capture(5)
    for i in range(3):
        a.replay()
        b.step(5)
        torch.cuda.synchronize()
        assert torch.equal(a.z, b.z) and torch.equal(a.h, b.h), i
    assert a.t == b.t == 15


@pytest.mark.parametrize("shape", [(2, 1024, 4, 3), (3, 1000, 16, 3), (2, 1100, 8, 2), (2, 1100, 24, 2),
                                   (2, 300, 64, 5)])
def test_fallback_finalize_steps_match_oracle(ref, mods, shape):
    """Steps at FFT lengths 2048 and 4096 (k_step2: a row over 256-chip
    blocks, one lane per chip, 4 and 16 logit levels per lane, partner
    spectra by k_rowspec; k_final with two chips per thread at 4096 when a
    chip has more than 16 logit levels) and with more logit levels per lane
    than k_step holds (k_final) against the oracle."""
    nat, optim, _ = mods
    M, N, L, F = shape
    prob = I.make_problem(M, N, L, F, p=16.0)
    opt = I.make_opt(total_iters=10, T0=1.0, T1=0.5)
    print(f"[gpu] fallback finalize M={M} N={N} L={L} F={F}", flush=True)
    run = optim.SQNGD([prob], opt, seeds=[5])
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


@pytest.mark.parametrize("schedule", ["throughput", "split8"])
def test_steps_at_fft_length_1024_match_oracle(ref, mods, schedule):
    """Two iterations of one M=2 N=512 design (FFT length 1024: the partner
    spectra that k_prep and k_step compute with one wave are stored in the
    throughput pass's two-wave layout, which both pass variants read)."""
    nat, optim, _ = mods
    prob = I.make_problem(2, 512, 4, 5, p=16.0)
    opt = I.make_opt(total_iters=10, T0=1.0, T1=0.5)
    sched = nat.SCHED_THROUGHPUT if schedule == "throughput" else nat.SCHED_SPLIT8
    print(f"[gpu] steps at FFT length 1024, {schedule}", flush=True)
    run = optim.SQNGD([prob], opt, seeds=[8], schedule=sched)
    s0 = run.numpy_state(0)
    run.step(2)
    torch.cuda.synchronize()
    s1 = run.numpy_state(0)
    z, h, state = s0["z"], s0["h"], s0["state"]
    for t in range(2):
        z, h, state, sta, stb = ref.step(prob, opt, z, h, state, t)
    assert _rel(s1["h"], h) <= 1e-4, _rel(s1["h"], h)
    assert _rel(s1["z"], z) <= 1e-4, _rel(s1["z"], z)
    sa, sb = run.step_stats()
    assert abs(sb[0]["loss"] - stb["loss"]) <= 1e-4 * stb["loss"]


def test_correlation_only_steps_match_oracle(ref, mods):
    """Correlation-only design (one Doppler bin at nu = 0, the paper's
    correlation experiments): two steps of a batch of two M=3 N=200 designs
    against the oracle."""
    nat, optim, _ = mods
    prob = I.make_problem(3, 200, 4, 1, nu_min=0.0, nu_max=0.0, p=16.0)
    opt = I.make_opt(total_iters=10, T0=1.0, T1=0.5)
    print("[gpu] correlation-only M=3 N=200 F=1", flush=True)
    run = optim.SQNGD([prob, prob], opt, seeds=[6, 7])
    s0 = [run.numpy_state(i) for i in range(2)]
    run.step(2)
    torch.cuda.synchronize()
    for i in range(2):
        s1 = run.numpy_state(i)
        z, h, state = s0[i]["z"], s0[i]["h"], s0[i]["state"]
        for t in range(2):
            z, h, state, sta, stb = ref.step(prob, opt, z, h, state, t)
        assert _rel(s1["h"], h) <= 1e-4, (i, _rel(s1["h"], h))
        assert _rel(s1["z"], z) <= 1e-4, (i, _rel(s1["z"], z))


def test_mixed_batch_steps_match_oracle(ref, mods):
    """One batch whose FFT-length groups finalize in different kernels (k_step
    for the short ones, k_final for the length-2048 one), several problems per
    group: every problem's two iterations against the oracle's."""
    nat, optim, _ = mods
    probs = [I.make_problem(2, 64, 4, 5, p=8.0), I.make_problem(3, 200, 8, 3, p=16.0),
             I.make_problem(2, 1024, 4, 2, p=16.0), I.make_problem(2, 60, 8, 4, p=8.0, sq_mode=I.PHASOR_MEAN)]
    opt = I.make_opt(total_iters=10, T0=1.0, T1=0.5)
    print("[gpu] mixed batch steps", flush=True)
    run = optim.SQNGD(probs, opt, seeds=[31, 32, 33, 34])
    s0 = [run.numpy_state(i) for i in range(len(probs))]
    run.step(2)
    torch.cuda.synchronize()
    assert run.t == 2
    for i, prob in enumerate(probs):
        s1 = run.numpy_state(i)
        z, h, state = s0[i]["z"], s0[i]["h"], s0[i]["state"]
        for t in range(2):
            z, h, state, _, _ = ref.step(prob, opt, z, h, state, t)
        assert _rel(s1["h"], h) <= 1e-4, (i, _rel(s1["h"], h))
        assert _rel(s1["z"], z) <= 1e-4, (i, _rel(s1["z"], z))


@pytest.mark.parametrize("layout", ["aligned", "misaligned"])
def test_step_logit_access_paths_match_oracle(ref, mods, layout):
    """k_step and k_step2 with one lane per chip (FFT lengths 1024, 2048) move a chip's
    logits and moments as 16-byte vectors only when L is a multiple of 4 and
    the rows are 16-byte aligned. 'aligned': two problems that take the
    vector path (L = 8 and 4); 'misaligned': a first problem of 101 x 3
    logits shifts the offsets of an L = 8 problem off 16 bytes, and an L = 5
    problem takes the scalar path by its L. Two iterations of every problem
    against the oracle's."""
    nat, optim, _ = mods
    if layout == "aligned":
        probs = [I.make_problem(2, 1000, 8, 2, p=16.0), I.make_problem(2, 400, 4, 3, p=16.0)]
    else:
        probs = [I.make_problem(1, 101, 3, 2, p=8.0), I.make_problem(2, 1000, 8, 2, p=16.0),
                 I.make_problem(2, 900, 5, 2, p=16.0)]
    opt = I.make_opt(total_iters=10, T0=1.0, T1=0.5)
    print(f"[gpu] step logit access, {layout}", flush=True)
    run = optim.SQNGD(probs, opt, seeds=list(range(40, 40 + len(probs))))
    s0 = [run.numpy_state(i) for i in range(len(probs))]
    run.step(2)
    torch.cuda.synchronize()
    for i, prob in enumerate(probs):
        s1 = run.numpy_state(i)
        z, h, state = s0[i]["z"], s0[i]["h"], s0[i]["state"]
        for t in range(2):
            z, h, state, _, _ = ref.step(prob, opt, z, h, state, t)
        assert _rel(s1["h"], h) <= 1e-4, (layout, i, _rel(s1["h"], h))
        assert _rel(s1["z"], z) <= 1e-4, (layout, i, _rel(s1["z"], z))
        assert _rel(s1["state"]["mz"], state["mz"]) <= 1e-3, (layout, i)
        assert _rel(s1["state"]["vz"], state["vz"]) <= 1e-3, (layout, i)


@pytest.mark.parametrize("layout", ["aligned", "misaligned"])
def test_row_split_step_at_fft_length_4096_matches_oracle(ref, mods, layout):
    """k_step2 (FFT length 4096, each row over blocks of 256 chips, the row's
    last block summing the products and projecting the filter row) in a
    batch with another FFT-length group, two filter and two logit steps per
    iteration (every next-pass preparation the chaining uses), three
    iterations against the oracle's. 'aligned': N = 2048 (eight blocks per
    row, the most) beside N = 1100 (five; its other three blocks exit),
    logits moved as 16-byte vectors (L = 4 and 8); 'misaligned': a first
    problem of 101 x 3 logits shifts the rows off 16 bytes, and L = 6 takes
    the scalar path by its L."""
    nat, optim, _ = mods
    if layout == "aligned":
        probs = [I.make_problem(2, 2048, 4, 2, p=16.0), I.make_problem(2, 1100, 8, 2, p=16.0),
                 I.make_problem(2, 200, 4, 3, p=8.0)]
    else:
        probs = [I.make_problem(1, 101, 3, 2, p=8.0), I.make_problem(2, 1200, 8, 2, p=16.0),
                 I.make_problem(3, 1030, 6, 2, p=16.0, sq_mode=I.PHASOR_MEAN)]
    opt = I.make_opt(n_h=2, n_x=2, total_iters=20, T0=1.0, T1=0.3)
    print(f"[gpu] row-split step at 4096, {layout}", flush=True)
    run = optim.SQNGD(probs, opt, seeds=list(range(60, 60 + len(probs))))
    s0 = [run.numpy_state(i) for i in range(len(probs))]
    iters = 3
    run.step(iters)
    torch.cuda.synchronize()
    assert run.t == iters
    sa, sb = run.step_stats()
    for i, prob in enumerate(probs):
        s1 = run.numpy_state(i)
        z, h, state = s0[i]["z"], s0[i]["h"], s0[i]["state"]
        for t in range(iters):
            z, h, state, sta, stb = ref.step(prob, opt, z, h, state, t)
        assert _rel(s1["h"], h) <= 1e-4, (layout, i, _rel(s1["h"], h))
        assert _rel(s1["z"], z) <= 1e-4, (layout, i, _rel(s1["z"], z))
        assert _rel(s1["state"]["mz"], state["mz"]) <= 1e-3, (layout, i)
        assert _rel(s1["state"]["vz"], state["vz"]) <= 1e-3, (layout, i)
        assert abs(sa[i]["loss"] - sta["loss"]) <= 1e-4 * sta["loss"], (layout, i)
        assert abs(sb[i]["loss"] - stb["loss"]) <= 1e-4 * stb["loss"], (layout, i)


@pytest.mark.parametrize("N", [1000, 999])
def test_wide_gradient_reduction_steps_match_oracle(ref, mods, N):
    """A group large enough (64 rows of FFT length 2048) for k_grad's one
    lane per chip (each wave reads 64 consecutive chips of a partial row),
    at an even and an odd N. Two iterations of 32 designs; three of them
    against the oracle's."""
    nat, optim, _ = mods
    prob = I.make_problem(2, N, 4, 2, p=16.0)
    opt = I.make_opt(total_iters=10, T0=1.0, T1=0.5)
    print(f"[gpu] wide gradient reduction N={N}", flush=True)
    run = optim.SQNGD([prob] * 32, opt, seeds=list(range(70, 102)))
    picks = (0, 17, 31)
    s0 = {i: run.numpy_state(i) for i in picks}
    run.step(2)
    torch.cuda.synchronize()
    sa, sb = run.step_stats()
    for i in picks:
        s1 = run.numpy_state(i)
        z, h, state = s0[i]["z"], s0[i]["h"], s0[i]["state"]
        for t in range(2):
            z, h, state, sta, stb = ref.step(prob, opt, z, h, state, t)
        assert _rel(s1["h"], h) <= 1e-4, (N, i, _rel(s1["h"], h))
        assert _rel(s1["z"], z) <= 1e-4, (N, i, _rel(s1["z"], z))
        assert abs(sa[i]["loss"] - sta["loss"]) <= 1e-4 * sta["loss"], (N, i)
        assert abs(sb[i]["loss"] - stb["loss"]) <= 1e-4 * stb["loss"], (N, i)


def test_row_split_step_in_two_launches_matches_oracle(ref, mods):
    """k_step2 for a launch of more than 96 blocks (12 designs of two rows,
    five blocks per row): the blocks write their partial products and
    k_step2_rows finishes each row in a second launch. Three iterations of
    two filter and two logit steps; two designs against the oracle's."""
    nat, optim, _ = mods
    prob = I.make_problem(2, 1100, 4, 2, p=16.0)
    opt = I.make_opt(n_h=2, n_x=2, total_iters=20, T0=1.0, T1=0.3)
    print("[gpu] row-split step in two launches", flush=True)
    run = optim.SQNGD([prob] * 12, opt, seeds=list(range(110, 122)))
    picks = (0, 11)
    s0 = {i: run.numpy_state(i) for i in picks}
    run.step(3)
    torch.cuda.synchronize()
    sa, sb = run.step_stats()
    for i in picks:
        s1 = run.numpy_state(i)
        z, h, state = s0[i]["z"], s0[i]["h"], s0[i]["state"]
        for t in range(3):
            z, h, state, sta, stb = ref.step(prob, opt, z, h, state, t)
        assert _rel(s1["h"], h) <= 1e-4, (i, _rel(s1["h"], h))
        assert _rel(s1["z"], z) <= 1e-4, (i, _rel(s1["z"], z))
        assert abs(sa[i]["loss"] - sta["loss"]) <= 1e-4 * sta["loss"], i
        assert abs(sb[i]["loss"] - stb["loss"]) <= 1e-4 * stb["loss"], i


def test_row_split_step_skips_nonfinite_row(mods):
    """k_step2: a NaN logit (chip 1050, the fifth of the row's five blocks)
    makes the logit step's loss non-finite; every block then leaves its
    logits unchanged."""
    nat, optim, _ = mods
    prob = I.make_problem(2, 1100, 8, 2, p=16.0)
    opt = I.make_opt(total_iters=10, T0=1.0, T1=0.5)
    print("[gpu] row-split step, non-finite", flush=True)
    run = optim.SQNGD([prob], opt, seeds=[4])
    run.z[8 * 1050 + 3] = float("nan")   # chip (0, 1050)
    z_before = run.z.clone()
    run.step()
    torch.cuda.synchronize()
    sa, sb = run.step_stats()
    assert sb[0]["nonfinite"] == 1
    assert sa[0]["nonfinite"] == 0
    assert torch.equal(torch.nan_to_num(run.z, nan=7.0), torch.nan_to_num(z_before, nan=7.0))
    assert torch.isfinite(run.h).all()


def test_subset_continues_bitwise(mods):
    """A sub-batch built from a running batch continues exactly as the batch
    does when both make the same calls (a call's first evaluation is prepared
    by k_prep, later ones by the finalize kernel, whose sums run in another
    order, so only equal call structures are bitwise comparable)."""
    nat, optim, _ = mods
    c = I.config("m2n64")
    print("[gpu] subset continuation", flush=True)
    a = optim.SQNGD([c["problem"]] * 3, c["opt"], seeds=[5, 6, 7], schedule=nat.SCHED_THROUGHPUT)
    a.run(6, use_graph=False)
    sub = a.subset([0, 2])
    a.run(6, use_graph=False)
    sub.run(6, use_graph=False)
    torch.cuda.synchronize()
    assert sub.t == a.t == 12
    for j, i in enumerate([0, 2]):
        assert torch.equal(sub.batch.unpack_z(sub.z, j), a.batch.unpack_z(a.z, i)), i
        assert torch.equal(sub.batch.unpack_w(sub.h, j), a.batch.unpack_w(a.h, i)), i
        assert torch.equal(sub.batch.unpack_adam(sub.adam, j), a.batch.unpack_adam(a.adam, i)), i


def test_stopping_rule_run(ref, mods):
    """optimise() with the stopping rule: each design stops where its own WPSL
    history says, its returned state is the state a plain run reaches at that
    iteration, and its hard statistics match the oracle's."""
    nat, optim, _ = mods
    c = I.config("m2n64")
    prob, opt = c["problem"], c["opt"]
    seeds = [11, 12, 13, 14]
    print("[gpu] stopping rule, 4 designs M=2 N=64", flush=True)
    res = optim.optimise([prob] * 4, opt, seeds=seeds, max_iters=120, check_every=10, patience=1,
                         min_gain_db=1.0, schedule=nat.SCHED_THROUGHPUT)
    stops = [d["stop_iter"] for d in res["designs"]]
    print("stop iterations", stops)
    assert any(s < 120 for s in stops)
    for i, d in enumerate(res["designs"]):
        hist = d["wpsl_db_history"]
        assert len(hist) == -(-d["stop_iter"] // 10)
        rule = optim.StopRule(1, patience=1, min_gain_db=1.0)
        fired = [bool(rule.update([0], [w])) for w in hist]
        assert fired[-1] or d["stop_iter"] == 120
        assert not any(fired[:-1])
        assert d["stats"]["pslr_db"] == hist[-1]
        # the same design alone, run for the same number of iterations
        plain = optim.SQNGD([prob], opt, seeds=[seeds[i]], schedule=nat.SCHED_THROUGHPUT)
        plain.run(d["stop_iter"], use_graph=False)
        torch.cuda.synchronize()
        assert np.array_equal(plain.batch.unpack_z(plain.z, 0).cpu().numpy(), d["z"]), i
        assert np.array_equal(plain.batch.unpack_w(plain.h, 0).cpu().numpy(), d["h"]), i
        assert np.array_equal(d["idx"], ref.hard_indices(d["z"].astype(np.float64)))
        st = ref.evaluate(ref.hard_waveform(d["z"].astype(np.float64)), d["h"].astype(np.complex128),
                          prob, False)[0]
        assert abs(d["stats"]["pslr_db"] - st["pslr_db"]) <= 0.05


@pytest.mark.parametrize("N,F,L", [(256, 129, 8), (256, 200, 8), (512, 33, 4)])
def test_fused_finalize_steps_match_oracle(ref, mods, N, F, L):
    """A batch of 32 M=4 designs (128 rows, at most 4 logit levels per lane:
    k_step reduces the gradient rows itself, in one load round per lane at
    N=256 F=129 and two at F=200; at N=512 the FFT length is 1024, where the
    finalize's one-wave spectra are stored in the multi-wave layout of the
    pass): two iterations of its first and last design against the oracle's."""
    nat, optim, _ = mods
    prob = I.make_problem(4, N, L, F, p=16.0)
    opt = I.make_opt(total_iters=10, T0=1.0, T1=0.5)
    print(f"[gpu] fused finalize 32 x M=4 N={N} F={F}", flush=True)
    run = optim.SQNGD([prob] * 32, opt, seeds=list(range(40, 72)), schedule=nat.SCHED_THROUGHPUT)
    s0 = [run.numpy_state(i) for i in (0, 31)]
    run.step(2)
    torch.cuda.synchronize()
    assert run.t == 2
    sa, sb = run.step_stats()
    for k, i in enumerate((0, 31)):
        s1 = run.numpy_state(i)
        z, h, state = s0[k]["z"], s0[k]["h"], s0[k]["state"]
        for t in range(2):
            z, h, state, sta, stb = ref.step(prob, opt, z, h, state, t)
        assert _rel(s1["h"], h) <= 1e-4, (i, _rel(s1["h"], h))
        assert _rel(s1["z"], z) <= 1e-4, (i, _rel(s1["z"], z))
        assert abs(sa[i]["loss"] - sta["loss"]) <= 1e-4 * sta["loss"]
        assert abs(sb[i]["loss"] - stb["loss"]) <= 1e-4 * stb["loss"]
        assert abs(sb[i]["pslr_db"] - stb["pslr_db"]) <= 0.05

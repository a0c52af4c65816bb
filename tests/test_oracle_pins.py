"""Pins of the FP64 oracle to facts that do not come from the oracle itself.

Each test checks the oracle against a library routine, a closed form, an
identity of the mathematics, a textbook example or brute force, chosen so that
a dropped term, a wrong sign, a wrong index or a swapped operand in the oracle
fails at least one of them.
"""
import itertools
import os

import numpy as np
import pytest

from paper_2604_25728_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_values(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                out[k] = float(v)
    return out


def _barker():
    rows = []
    with open(os.path.join(GOLDEN, "barker13.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([float(v) for v in line.split()])
    return np.array(rows[0]), np.array(rows[1])


def _rand_c(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ---------------------------------------------------------------- the AF (eq. 6)

def test_zero_doppler_is_numpy_correlate(ref):
    """At nu = 0 the AF is the aperiodic cross-correlation; numpy.correlate(a, v)[k]
    = sum_n a[n+k] conj(v[n]) gives A(tau) at k = -tau."""
    M, N, F = 3, 17, 5
    s, h = _rand_c((M, N), 1), _rand_c((M, N), 2)
    cube = ref.af_cube(s, h, F, -0.5, 0.5)
    f0 = F // 2
    assert abs(ref.doppler_grid(F, -0.5, 0.5)[f0]) < 1e-15
    for m in range(M):
        for l in range(M):
            lib = np.correlate(s[m], h[l], mode="full")[::-1]
            np.testing.assert_allclose(cube[m, l, f0], lib, rtol=0, atol=1e-12)


def test_mainlobe_is_inner_product(ref):
    """A_mm(0, 0) = h_m^H s_m (eq. 38), and = N for a unimodular matched pair."""
    M, N, F = 2, 32, 3
    s, h = _rand_c((M, N), 3), _rand_c((M, N), 4)
    cube = ref.af_cube(s, h, F, -0.25, 0.25)
    for m in range(M):
        assert abs(cube[m, m, 1, N - 1] - np.vdot(h[m], s[m])) < 1e-12
    u = np.exp(2j * np.pi * np.random.default_rng(5).random((M, N)))
    cube = ref.af_cube(u, u, F, -0.25, 0.25)
    assert abs(cube[0, 0, 1, N - 1] - N) < 1e-12


def test_cauchy_schwarz_bound(ref):
    M, N, F = 3, 24, 7
    s, h = _rand_c((M, N), 6), _rand_c((M, N), 7)
    cube = ref.af_cube(s, h, F, -1.5, 1.5)
    bound = np.linalg.norm(s, axis=1)[:, None, None, None] * np.linalg.norm(h, axis=1)[None, :, None, None]
    assert np.all(np.abs(cube) <= bound * (1 + 1e-12))


def test_delay_sum_factorises(ref):
    """sum_tau A(tau, nu) = (sum_n xh(n)) conj(sum_n h(n))."""
    M, N, F = 2, 19, 4
    s, h = _rand_c((M, N), 8), _rand_c((M, N), 9)
    nu = ref.doppler_grid(F, -0.7, 0.9)
    cube = ref.af_cube(s, h, F, -0.7, 0.9)
    n = np.arange(N)
    for m, l, f in itertools.product(range(M), range(M), range(F)):
        xh = s[m] * np.exp(2j * np.pi * n * nu[f] / N)
        assert abs(cube[m, l, f].sum() - xh.sum() * np.conj(h[l].sum())) < 1e-10


def test_parseval_per_doppler_bin(ref):
    """sum_tau |A|^2 = (1/P) sum_k |FFT(xh)_k|^2 |FFT(h)_k|^2 with P >= 2N-1 (numpy.fft)."""
    M, N, F = 2, 21, 3
    s, h = _rand_c((M, N), 10), _rand_c((M, N), 11)
    nu = ref.doppler_grid(F, -0.5, 0.5)
    cube = ref.af_cube(s, h, F, -0.5, 0.5)
    P = 64
    n = np.arange(N)
    for m, l, f in itertools.product(range(M), range(M), range(F)):
        X = np.fft.fft(s[m] * np.exp(2j * np.pi * n * nu[f] / N), P)
        H = np.fft.fft(h[l], P)
        lhs = (np.abs(cube[m, l, f]) ** 2).sum()
        rhs = (np.abs(X) ** 2 * np.abs(H) ** 2).sum() / P
        assert abs(lhs - rhs) < 1e-9 * rhs


def test_moyal_identity_integer_grid(ref):
    """On N integer Doppler bins sum_{tau,nu} |A|^2 = N |s|^2 |h|^2."""
    N = 16
    s, h = _rand_c((1, N), 12), _rand_c((1, N), 13)
    cube = ref.af_cube(s, h, N, 0.0, N - 1.0)
    lhs = (np.abs(cube) ** 2).sum()
    rhs = N * np.linalg.norm(s) ** 2 * np.linalg.norm(h) ** 2
    assert abs(lhs - rhs) < 1e-10 * rhs


def test_role_swap_symmetry(ref):
    """|A_{s,h}(tau, nu)| = |A_{h,s}(-tau, -nu)| on a symmetric Doppler grid."""
    M, N, F = 2, 15, 9
    s, h = _rand_c((M, N), 14), _rand_c((M, N), 15)
    a = np.abs(ref.af_cube(s, h, F, -0.8, 0.8))
    b = np.abs(ref.af_cube(h, s, F, -0.8, 0.8))
    for m, l in itertools.product(range(M), range(M)):
        np.testing.assert_allclose(a[m, l], b[l, m, ::-1, ::-1], rtol=1e-10, atol=1e-12)


def test_constant_sequence_dirichlet(ref):
    """For s = h = 1: |A(tau, nu)| = |sin(pi nu (N-|tau|)/N) / sin(pi nu / N)|, N - |tau| at nu = 0."""
    N, F = 20, 33
    one = np.ones((1, N))
    nu = ref.doppler_grid(F, -0.5, 0.5)
    cube = np.abs(ref.af_cube(one, one, F, -0.5, 0.5))[0, 0]
    tau = np.arange(-(N - 1), N)
    for f in range(F):
        if abs(nu[f]) < 1e-14:
            want = N - np.abs(tau)
        else:
            want = np.abs(np.sin(np.pi * nu[f] * (N - np.abs(tau)) / N) / np.sin(np.pi * nu[f] / N))
        np.testing.assert_allclose(cube[f], want, rtol=1e-10, atol=1e-10)


def test_barker13(ref):
    """Textbook Barker-13: autocorrelation 13, 0, 1, 0, 1, ...; PSL 1; PSLR = 20 log10(1/13)."""
    code, acf = _barker()
    g = _golden_values("closed_forms.txt")
    prob = I.make_problem(1, 13, 2, 1, nu_min=0.0, nu_max=0.0, p=8.0)
    s = code[None, :].astype(np.complex128)
    cube = ref.af_cube(s, s, 1, 0.0, 0.0)
    row = cube[0, 0, 0]
    np.testing.assert_allclose(row[12:], acf, atol=1e-12)
    np.testing.assert_allclose(row[:13], acf[::-1], atol=1e-12)
    st = ref.loss_stats(cube, s, s, prob)
    assert abs(st["psl_auto"] - 1.0) < 1e-12
    assert abs(st["pslr_db"] - g["pslr_barker13"]) < 1e-9
    assert st["psl_cross"] == 0.0  # M = 1: no cross pairs


def test_brute_force_binary_13(ref):
    """Over all 2^13 binary codes the best auto PSL (tau != 0) is 1, reached by Barker-13."""
    N = 13
    prob = I.make_problem(1, N, 2, 1, nu_min=0.0, nu_max=0.0, p=8.0)
    best = np.inf
    for bits in range(1 << (N - 1)):  # fix the first chip: PSL is invariant to a sign flip
        code = np.array([1.0] + [1.0 if (bits >> i) & 1 else -1.0 for i in range(N - 1)])
        s = code[None, :].astype(np.complex128)
        cube = ref.af_cube(s, s, 1, 0.0, 0.0)
        best = min(best, ref.loss_stats(cube, s, s, prob)["psl_auto"])
    assert abs(best - 1.0) < 1e-12


# ------------------------------------------------------- loss (eq. 7-10, 37-42, 48)

def test_snrl_closed_forms(ref):
    g = _golden_values("closed_forms.txt")
    M, N, F = 2, 32, 5
    u = np.exp(2j * np.pi * np.random.default_rng(16).random((M, N)))
    prob = I.make_problem(M, N, 4, F, p=8.0, snrl_target_db=0.5)
    st = ref.loss_stats(ref.af_cube(u, u, F, -0.5, 0.5), u, u, prob)
    assert abs(st["snrl_db_max"]) < 1e-12            # matched filter: no SNR loss (eq. 10)
    assert abs(st["p_min"] - 1.0) < 1e-12             # p_m = |h^H x| / N = 1 (eq. 38)
    assert abs(st["l_snrl"] - (1.0 - g["p_tar_0p5db"]) ** 2) < 1e-15  # eq. 39, 41
    # a scaled filter keeps the SNRL at 0 dB but changes p_m
    st2 = ref.loss_stats(ref.af_cube(u, 2 * u, F, -0.5, 0.5), u, 2 * u, prob)
    assert abs(st2["snrl_db_max"]) < 1e-12
    assert abs(st2["p_min"] - 2.0) < 1e-12
    # a filter rotated by a common phase loses nothing
    w = u * np.exp(1j * np.pi / 3)
    st3 = ref.loss_stats(ref.af_cube(u, w, F, -0.5, 0.5), u, w, prob)
    assert abs(st3["snrl_db_max"]) < 1e-12
    # a quarter of the chips flipped: |h^H x| = N/2, so SNRL = 10 log10(4)
    q = u.copy()
    q[:, : N // 4] *= -1
    st4 = ref.loss_stats(ref.af_cube(u, q, F, -0.5, 0.5), u, q, prob)
    assert abs(st4["snrl_db_max"] - 10 * np.log10(4.0)) < 1e-10
    assert abs(st4["p_min"] - 0.5) < 1e-12


def test_lp_limits_and_parseval(ref):
    """L_p decreases in p towards max a = PSL/N; L_2^2 N^2 = sum |A|^2 minus the excluded cells."""
    M, N, F = 2, 16, 5
    s, h = _rand_c((M, N), 17), _rand_c((M, N), 18)
    cube = ref.af_cube(s, h, F, -0.5, 0.5)
    lps = []
    for p in [2, 4, 8, 16, 64, 256, 1024]:
        prob = I.make_problem(M, N, 4, F, p=float(p))
        lps.append(ref.loss_stats(cube, s, h, prob)["lp"])
    st = ref.loss_stats(cube, s, h, I.make_problem(M, N, 4, F, p=8.0))
    amax = max(st["psl_auto"], st["psl_cross"]) / N
    assert all(a >= b for a, b in zip(lps, lps[1:]))
    assert lps[-1] >= amax and lps[-1] < amax * 1.01
    # p = 2 against an FFT (Parseval) total over all cells minus the auto tau = 0 cuts
    nu = ref.doppler_grid(F, -0.5, 0.5)
    n = np.arange(N)
    total = 0.0
    for m, l, f in itertools.product(range(M), range(M), range(F)):
        X = np.fft.fft(s[m] * np.exp(2j * np.pi * n * nu[f] / N), 64)
        H = np.fft.fft(h[l], 64)
        total += (np.abs(X) ** 2 * np.abs(H) ** 2).sum() / 64
        if m == l:
            total -= abs(np.vdot(h[l], s[m] * np.exp(2j * np.pi * n * nu[f] / N))) ** 2
    assert abs(lps[0] ** 2 * N * N - total) < 1e-9 * total


def test_delay_window(ref):
    """Cells outside [tau_lo, tau_hi] do not count."""
    M, N, F = 2, 12, 3
    s, h = _rand_c((M, N), 19), _rand_c((M, N), 20)
    cube = ref.af_cube(s, h, F, -0.5, 0.5)
    prob = I.make_problem(M, N, 4, F, p=4.0, tau_lo=-3, tau_hi=5)
    st = ref.loss_stats(cube, s, h, prob)
    a = np.abs(cube)
    tau = np.arange(-(N - 1), N)
    win = (tau >= -3) & (tau <= 5)
    auto = max(a[m, m, :, win & (tau != 0)].max() for m in range(M))
    cross = max(a[m, l, :, win].max() for m in range(M) for l in range(M) if m != l)
    assert abs(st["psl_auto"] - auto) < 1e-12 and abs(st["psl_cross"] - cross) < 1e-12


# ------------------------------------------------------------------- gradients

def _fd_check(ref, s, h, prob, coords, step=1e-6):
    st, gs, gh = ref.evaluate(s, h, prob)
    for which, m, n in coords:
        for unit in (1.0, 1j):
            sp, sm, hp, hm = s.copy(), s.copy(), h.copy(), h.copy()
            if which == "s":
                sp[m, n] += step * unit
                sm[m, n] -= step * unit
            else:
                hp[m, n] += step * unit
                hm[m, n] -= step * unit
            Lp = ref.evaluate(sp, hp, prob, want_grads=False)[0]["loss"]
            Lm = ref.evaluate(sm, hm, prob, want_grads=False)[0]["loss"]
            fd = (Lp - Lm) / (2 * step)
            g = (gs if which == "s" else gh)[m, n]
            an = g.real if unit == 1.0 else g.imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)) + 1e-8, (which, m, n, unit, fd, an)


def test_gradients_central_differences(ref):
    M, N, F = 2, 8, 5
    s, h = _rand_c((M, N), 21), _rand_c((M, N), 22)
    prob = I.make_problem(M, N, 4, F, nu_min=-0.6, nu_max=0.4, p=8.0, w_snrl=0.7, w_psl=1.3,
                          tau_lo=-5, tau_hi=6)
    rng = np.random.default_rng(23)
    coords = [(w, int(rng.integers(M)), int(rng.integers(N))) for w in ("s", "h") for _ in range(6)]
    _fd_check(ref, s, h, prob, coords)


def test_gradients_against_torch_fft_autograd(ref):
    """Independent route: torch complex128 autograd through the FFT correlation of eq. 36."""
    torch = pytest.importorskip("torch")
    M, N, F = 3, 10, 6
    s0, h0 = _rand_c((M, N), 24), _rand_c((M, N), 25)
    prob = I.make_problem(M, N, 4, F, nu_min=-1.0, nu_max=0.5, p=6.0, w_snrl=0.5)
    st, gs, gh = ref.evaluate(s0, h0, prob)
    s = torch.tensor(s0, dtype=torch.complex128, requires_grad=True)
    h = torch.tensor(h0, dtype=torch.complex128, requires_grad=True)
    P = 32
    nu = torch.tensor(ref.doppler_grid(F, -1.0, 0.5))
    n = torch.arange(N, dtype=torch.float64)
    mod = torch.exp(2j * torch.pi * n[None, :] * nu[:, None] / N)          # [F][N]
    X = torch.fft.fft(s[:, None, :] * mod[None], n=P)                        # [M][F][P]
    H = torch.fft.fft(h, n=P)                                                # [M][P]
    r = torch.fft.ifft(X[:, None, :, :] * torch.conj(H)[None, :, None, :])  # [M][M][F][P]
    tau = torch.arange(-(N - 1), N)
    A = r[..., (-tau) % P]                                                   # A(tau) = r[-tau mod P]
    a = A.abs() / N
    mask = torch.ones_like(a, dtype=torch.bool)
    for m in range(M):
        mask[m, m, :, N - 1] = False
    lp = (a[mask] ** prob["p"]).sum() ** (1.0 / prob["p"])
    c = (torch.conj(h) * s).sum(dim=1)
    p_tar = 10 ** (-prob["snrl_target_db"] / 20)
    l_snrl = ((c.abs() / N - p_tar) ** 2).mean()
    loss = prob["w_psl"] * lp + prob["w_snrl"] * l_snrl
    loss.backward()
    assert abs(loss.item() - st["loss"]) < 1e-12
    np.testing.assert_allclose(s.grad.numpy(), gs, rtol=0, atol=1e-10 * np.abs(gs).max())
    np.testing.assert_allclose(h.grad.numpy(), gh, rtol=0, atol=1e-10 * np.abs(gh).max())


def test_mainlobe_mask_against_torch_fft_autograd(ref):
    """auto_mask = 1 (only the Doppler-mainlobe cells |nu| < 1 of an auto pair's
    tau = 0 cut leave the region): loss, PSLs, peak and both gradients against
    torch complex128 autograd through the FFT correlation of eq. 36, with the
    grid and the mask built here (numpy linspace), not by the oracle."""
    torch = pytest.importorskip("torch")
    M, N, F = 3, 10, 11
    s0, h0 = _rand_c((M, N), 54), _rand_c((M, N), 55)
    # unimodular waveforms with h = s: the cut's cells at nu = +-1.5, +-2.5
    # are Dirichlet sidelobes, larger than most delay sidelobes
    s0 = np.exp(1j * np.angle(s0))
    h0 = s0 + 0.1 * h0
    prob = I.make_problem(M, N, 4, F, nu_min=-2.5, nu_max=2.5, p=6.0, w_snrl=0.5, auto_mask=1)
    st, gs, gh = ref.evaluate(s0, h0, prob)
    s = torch.tensor(s0, dtype=torch.complex128, requires_grad=True)
    h = torch.tensor(h0, dtype=torch.complex128, requires_grad=True)
    P = 32
    nu_np = np.linspace(-2.5, 2.5, F)
    nu = torch.tensor(nu_np)
    n = torch.arange(N, dtype=torch.float64)
    mod = torch.exp(2j * torch.pi * n[None, :] * nu[:, None] / N)
    X = torch.fft.fft(s[:, None, :] * mod[None], n=P)
    H = torch.fft.fft(h, n=P)
    r = torch.fft.ifft(X[:, None, :, :] * torch.conj(H)[None, :, None, :])
    tau = torch.arange(-(N - 1), N)
    A = r[..., (-tau) % P]
    a = A.abs() / N
    mask = torch.ones_like(a, dtype=torch.bool)
    main = torch.tensor(np.abs(nu_np) < 1.0)
    assert int(main.sum()) == 3  # nu = -0.5, 0, 0.5
    for m in range(M):
        mask[m, m, main, N - 1] = False
    lp = (a[mask] ** prob["p"]).sum() ** (1.0 / prob["p"])
    c = (torch.conj(h) * s).sum(dim=1)
    p_tar = 10 ** (-prob["snrl_target_db"] / 20)
    loss = prob["w_psl"] * lp + prob["w_snrl"] * ((c.abs() / N - p_tar) ** 2).mean()
    loss.backward()
    assert abs(loss.item() - st["loss"]) < 1e-12
    an = a.detach().numpy() * N
    mk = mask.numpy()
    auto = max(an[m, m][mk[m, m]].max() for m in range(M))
    cross = max(an[m, l].max() for m in range(M) for l in range(M) if m != l)
    assert abs(st["psl_auto"] - auto) < 1e-12 and abs(st["psl_cross"] - cross) < 1e-12
    v = np.where(mk, an, -1.0)
    m_, l_, f_, k_ = np.unravel_index(int(np.argmax(v)), v.shape)
    assert tuple(st["arg"]) == (m_, l_, k_ - (N - 1), f_)
    np.testing.assert_allclose(s.grad.numpy(), gs, rtol=0, atol=1e-10 * np.abs(gs).max())
    np.testing.assert_allclose(h.grad.numpy(), gh, rtol=0, atol=1e-10 * np.abs(gh).max())
    # the cut's Doppler sidelobes do enter: the paper's rule gives a smaller loss
    st0 = ref.evaluate(s0, h0, dict(prob, auto_mask=0), False)[0]
    assert st0["lp"] < st["lp"] - 1e-6
    # a span inside the mainlobe: both rules select the same cells
    inner = dict(prob, nu_min=-0.5, nu_max=0.5)
    st1, gs1, gh1 = ref.evaluate(s0, h0, inner)
    st2, gs2, gh2 = ref.evaluate(s0, h0, dict(inner, auto_mask=0))
    assert st1["loss"] == st2["loss"] and np.array_equal(gs1, gs2) and np.array_equal(gh1, gh2)


@pytest.mark.parametrize("mode", [I.PHASE_MEAN, I.PHASOR_MEAN])
def test_logit_chain_central_differences(ref, mode):
    M, N, L, F = 2, 8, 4, 3
    prob = I.make_problem(M, N, L, F, p=8.0, sq_mode=mode)
    z = np.random.default_rng(26).standard_normal((M, N, L))
    h = _rand_c((M, N), 27)
    T = 0.7
    s = ref.soft_waveform(z, T, mode)
    _, gs, _ = ref.evaluate(s, h, prob)
    gz = ref.logit_grad(z, T, gs, mode)
    rng = np.random.default_rng(28)
    for _ in range(8):
        m, n, l = int(rng.integers(M)), int(rng.integers(N)), int(rng.integers(L))
        zp, zm = z.copy(), z.copy()
        zp[m, n, l] += 1e-6
        zm[m, n, l] -= 1e-6
        Lp = ref.evaluate(ref.soft_waveform(zp, T, mode), h, prob, False)[0]["loss"]
        Lm = ref.evaluate(ref.soft_waveform(zm, T, mode), h, prob, False)[0]["loss"]
        fd = (Lp - Lm) / 2e-6
        assert abs(fd - gz[m, n, l]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9


# ------------------------------------------------------ quantisers and optimiser

def test_hard_quantiser(ref):
    z = np.random.default_rng(29).standard_normal((3, 40, 8))
    z[0, 0, :] = 1.0          # all tied -> level 0
    z[1, 5, [2, 6]] = 9.0     # tie between 2 and 6 -> 2
    idx = ref.hard_indices(z)
    np.testing.assert_array_equal(idx, np.argmax(z, axis=-1))  # numpy: first maximum
    assert idx[0, 0] == 0 and idx[1, 5] == 2
    x = ref.hard_waveform(z)
    np.testing.assert_allclose(np.abs(x), 1.0, atol=1e-15)
    np.testing.assert_allclose(x, np.exp(2j * np.pi * idx / 8), atol=1e-15)


def test_soft_waveform_limits(ref):
    z = np.random.default_rng(30).standard_normal((2, 50, 8))
    s = ref.soft_waveform(z, 1.0, I.PHASE_MEAN)
    np.testing.assert_allclose(np.abs(s), 1.0, atol=1e-14)  # phase-mean is unimodular
    srt = np.sort(z, axis=-1)
    clear = (srt[..., -1] - srt[..., -2]) > 0.05
    cold = ref.soft_waveform(z, 1e-3, I.PHASE_MEAN)
    np.testing.assert_allclose(cold[clear], ref.hard_waveform(z)[clear], atol=1e-9)
    cold2 = ref.soft_waveform(z, 1e-3, I.PHASOR_MEAN)
    np.testing.assert_allclose(cold2[clear], ref.hard_waveform(z)[clear], atol=1e-9)
    hot = ref.soft_waveform(np.zeros((1, 3, 8)), 1.0, I.PHASOR_MEAN)
    np.testing.assert_allclose(hot, 0.0, atol=1e-15)  # uniform weights: phasors cancel


def test_adam_matches_torch(ref):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(31)
    p0 = rng.standard_normal(20)
    grads = [rng.standard_normal(20) for _ in range(7)]
    tp = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=3e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(20), np.zeros(20)
    for t, g in enumerate(grads, start=1):
        opt.zero_grad()
        tp.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = ref.adam(p, g, m, v, t, 3e-2, 0.9, 0.999, 1e-8)
        np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-14, atol=1e-15)


def test_projection(ref):
    h = _rand_c((3, 33), 32)
    ph = ref.project(h)
    np.testing.assert_allclose((np.abs(ph) ** 2).sum(axis=1), 33.0, rtol=1e-14)
    np.testing.assert_allclose(ref.project(ph), ph, rtol=1e-14)
    # direction kept
    np.testing.assert_allclose(ph / np.linalg.norm(ph, axis=1, keepdims=True),
                               h / np.linalg.norm(h, axis=1, keepdims=True), rtol=1e-13)


def test_temperature_schedule(ref):
    assert ref.temperature(0, 1.0, 0.05, 2000) == 1.0
    assert abs(ref.temperature(1999, 1.0, 0.05, 2000) - 0.05) < 1e-15
    r = [ref.temperature(t + 1, 1.0, 0.05, 2000) / ref.temperature(t, 1.0, 0.05, 2000)
         for t in (0, 500, 1500)]
    np.testing.assert_allclose(r, 0.05 ** (1 / 1999), rtol=1e-13)
    assert ref.temperature(5000, 1.0, 0.05, 2000) == pytest.approx(0.05)
    assert ref.temperature(3, 0.7, 0.1, 1) == 0.7


def test_step_invariants_and_improvement(ref):
    """Filters stay on the energy sphere (eq. 31-32); a short M=2 N=64 run lowers the loss."""
    cfg = I.config("m2n64")
    prob, opt = cfg["problem"], cfg["opt"]
    z = I.logits(prob["M"], prob["N"], prob["L"], 0).astype(np.float64)
    h = ref.matched_init(z)
    st0 = ref.evaluate(ref.hard_waveform(z), h, prob, False)[0]
    state = ref.new_state(prob["M"], prob["N"], prob["L"])
    for t in range(40):
        z, h, state, sa, sb = ref.step(prob, opt, z, h, state, t)
        np.testing.assert_allclose((np.abs(h) ** 2).sum(axis=1), prob["N"], rtol=1e-12)
    st1 = ref.evaluate(ref.hard_waveform(z), h, prob, False)[0]
    assert st1["loss"] < st0["loss"]
    assert sa is not None and sb is not None


# ------------------------------------------------- ROI weights w(tau, f) (eq. 8-9)

def _weights(F, N, seed, lo=0.3, hi=2.0):
    return np.random.default_rng(seed).uniform(lo, hi, size=(F, 2 * N - 1))


def test_weights_of_one_and_indicator_windows(ref):
    """w = 1 gives the unweighted statistics; a 0/1 table equal to a delay
    window gives the window's statistics (the window is eq. 8-9 with an
    indicator weight)."""
    M, N, F = 2, 12, 4
    s, h = _rand_c((M, N), 41), _rand_c((M, N), 42)
    cube = ref.af_cube(s, h, F, -0.5, 0.5)
    base = I.make_problem(M, N, 4, F, p=6.0)
    st0 = ref.loss_stats(cube, s, h, base)
    st1 = ref.loss_stats(cube, s, h, dict(base, roi_w=np.ones((F, 2 * N - 1))))
    for k in ("loss", "lp", "psl_auto", "psl_cross"):
        assert st1[k] == st0[k], k
    tau = np.arange(-(N - 1), N)
    ind = np.tile(((tau >= -4) & (tau <= 7)).astype(float), (F, 1))
    stw = ref.loss_stats(cube, s, h, dict(base, roi_w=ind))
    stn = ref.loss_stats(cube, s, h, dict(base, tau_lo=-4, tau_hi=7))
    for k in ("lp", "psl_auto", "psl_cross"):
        assert abs(stw[k] - stn[k]) <= 1e-12 * stn[k], k


def test_weighted_psl_and_norm_by_brute_force(ref):
    """PSL and L_p with random weights against a numpy scan of the cube."""
    M, N, F, p = 3, 9, 5, 5.0
    s, h = _rand_c((M, N), 43), _rand_c((M, N), 44)
    cube = ref.af_cube(s, h, F, -0.7, 0.3)
    wt = _weights(F, N, 45)
    st = ref.loss_stats(cube, s, h, dict(I.make_problem(M, N, 4, F, p=p), roi_w=wt))
    aw = np.abs(cube) * wt[None, None]
    auto_mask = np.ones(2 * N - 1, bool)
    auto_mask[N - 1] = False
    auto = max(aw[m, m][:, auto_mask].max() for m in range(M))
    cross = max(aw[m, l].max() for m in range(M) for l in range(M) if m != l)
    cells = [aw[m, l][:, auto_mask] if m == l else aw[m, l] for m in range(M) for l in range(M)]
    lp = (sum(((c / N) ** p).sum() for c in cells)) ** (1 / p)
    assert abs(st["psl_auto"] - auto) < 1e-12 * auto and abs(st["psl_cross"] - cross) < 1e-12 * cross
    assert abs(st["lp"] - lp) < 1e-12 * lp


def test_weight_scaling(ref):
    """w -> c w scales L_p and both PSLs by c and the sidelobe part of the gradient by c."""
    M, N, F = 2, 10, 3
    s, h = _rand_c((M, N), 46), _rand_c((M, N), 47)
    wt = _weights(F, N, 48)
    prob = dict(I.make_problem(M, N, 4, F, p=8.0, w_snrl=0.0), roi_w=wt)
    st, gs, gh = ref.evaluate(s, h, prob)
    st3, gs3, gh3 = ref.evaluate(s, h, dict(prob, roi_w=3.0 * wt))
    for k in ("lp", "psl_auto", "psl_cross"):
        assert abs(st3[k] - 3.0 * st[k]) <= 1e-12 * st3[k], k
    assert np.abs(gs3 - 3.0 * gs).max() <= 1e-12 * np.abs(gs3).max()
    assert np.abs(gh3 - 3.0 * gh).max() <= 1e-12 * np.abs(gh3).max()


def test_weighted_gradients_central_differences(ref):
    M, N, F = 2, 8, 4
    s, h = _rand_c((M, N), 49), _rand_c((M, N), 50)
    prob = dict(I.make_problem(M, N, 4, F, nu_min=-0.4, nu_max=0.6, p=6.0, w_snrl=0.8, tau_lo=-6, tau_hi=5),
                roi_w=_weights(F, N, 51))
    rng = np.random.default_rng(52)
    coords = [(w, int(rng.integers(M)), int(rng.integers(N))) for w in ("s", "h") for _ in range(6)]
    _fd_check(ref, s, h, prob, coords)

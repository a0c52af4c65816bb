"""Wide Doppler spans (the paper's Table III reaches nu in [-N/2, N/2] = [-600,
600] at N = 1200, where the modulation phase n nu / N of eq. 33 holds up to
600 whole turns) against the FP64 oracle: statistics, peak location and both
gradients on a 25-bin sample of the span (integer and non-integer grids), and
sampled AF rows of the full integer grid (F = 1201).

Tolerances as in test_gpu_parity: AF cells within 1e-4 max|A|, loss 1e-4
relative, PSL / SNRL within 0.05 dB, gradients 1e-4 normwise."""
import numpy as np
import pytest
from helpers import check_peak

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


@pytest.mark.parametrize("span", [(-600.0, 600.0), (-599.3, 600.9)])
def test_wide_span_evaluation(ref, nat, span):
    """25 bins over the span: every bin far from nu = 0 (integer multiples of
    50 on the first grid, non-representable steps on the second)."""
    prob = I.make_problem(2, 1200, 16, 25, nu_min=span[0], nu_max=span[1], p=16.0)
    M, N, L = prob["M"], prob["N"], prob["L"]
    print(f"[gpu] wide span {span}", flush=True)
    z, h = I.logits(M, N, L, 90), I.complex_gaussian(M, N, 91)
    b = nat.Batch([prob])
    zt, ht = b.pack_z([z]), b.pack_w([h])
    stats_f, cube = b.af_forward(zt, ht, nat.WAVE_SOFT, cube=True)
    stats_b = b.new_stats()
    gz, gh, gs = b.af_backward(zt, ht, nat.WAVE_SOFT, want_s=True, stats=stats_b)
    torch.cuda.synchronize()
    s = ref.soft_waveform(z.astype(np.float64), prob["temperature"])
    hr = h.astype(np.complex128)
    cref = ref.af_cube(s, hr, prob["F"], prob["nu_min"], prob["nu_max"])
    st_ref = ref.loss_stats(cref, s, hr, prob)
    gs_ref, gh_ref = ref.grads(s, hr, prob, cref)
    c = b.unpack_cube(cube, 0).cpu().numpy()
    assert np.abs(c - cref).max() <= 1e-4 * np.abs(cref).max()
    for st in (nat.decode_stats(stats_f.cpu().numpy())[0], nat.decode_stats(stats_b.cpu().numpy())[0]):
        assert abs(st["loss"] - st_ref["loss"]) <= 1e-4 * st_ref["loss"], (st, st_ref)
        for k in ("psl_auto", "psl_cross"):
            assert abs(_db(st[k]) - _db(st_ref[k])) <= 0.05, (k, st[k], st_ref[k])
        assert abs(st["snrl_db_max"] - st_ref["snrl_db_max"]) <= 0.05
        check_peak(st, cref, prob)
    for m in range(M):
        assert _rel(gs.cpu().numpy().reshape(M, N)[m], gs_ref[m]) <= 1e-4, m
        assert _rel(gh.cpu().numpy().reshape(M, N)[m], gh_ref[m]) <= 1e-4, m
    gz_ref = ref.logit_grad(z.astype(np.float64), prob["temperature"], gs_ref)
    assert _rel(gz.cpu().numpy(), gz_ref) <= 1e-4


def test_full_integer_grid_sampled_rows(ref, nat):
    """Table III's widest grid at N = 1200: F = 1201 integer bins over
    [-600, 600]; AF rows at the span's ends, around nu = 0 and in between
    against the oracle's direct sums (hard waveforms, given filters)."""
    prob = I.make_problem(2, 1200, 16, 1201, nu_min=-600.0, nu_max=600.0, p=16.0)
    M, N, L, F = prob["M"], prob["N"], prob["L"], prob["F"]
    print("[gpu] wide span F=1201 sampled rows", flush=True)
    z, h = I.logits(M, N, L, 92), I.complex_gaussian(M, N, 93)
    b = nat.Batch([prob])
    zt, ht = b.pack_z([z]), b.pack_w([h])
    _, cube = b.af_forward(zt, ht, nat.WAVE_HARD, cube=True)
    torch.cuda.synchronize()
    x = ref.hard_waveform(z)
    hr = h.astype(np.complex128)
    c = b.unpack_cube(cube, 0)
    amax = float(c.abs().max().item())
    rows = [(0, 0, 0), (1, 1, F - 1), (0, 1, 600), (1, 0, 601), (0, 0, 599), (1, 1, 7), (0, 1, 1123), (1, 0, 318)]
    for m, l, f in rows:
        want = ref.af_row(x, hr, F, prob["nu_min"], prob["nu_max"], m, l, f)
        got = c[m, l, f].cpu().numpy()
        assert np.abs(got - want).max() <= 1e-4 * amax, (m, l, f, np.abs(got - want).max() / amax)

"""sqngd_af_backward_noalloc (the evaluation without a workspace, scratch in
the library's static per-GPU array) against sqngd_af_backward on the same
inputs: two calls in a row, the second with a smaller batch, so the second
runs on scratch that still holds the first call's plan and partials.
The two entry points run the same kernels, so their outputs must agree bit
for bit; the first call is also held to the oracle's tolerances (1e-4)."""
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


def _both(nat, probs, z, h, mode, s=None, want_z=True, want_s=True):
    b = nat.Batch(probs)
    st_w, st_n = b.new_stats(), b.new_stats()
    with_ws = b.af_backward(z, h, mode, s_given=s, want_z=want_z, want_h=True, want_s=want_s, stats=st_w)
    no_ws = nat.af_backward_noalloc(probs, z, h, mode, s_given=s, want_z=want_z, want_h=True, want_s=want_s,
                                    stats=st_n)
    torch.cuda.synchronize()
    for a, c in zip(with_ws, no_ws):
        assert (a is None) == (c is None)
        if a is not None:
            assert torch.equal(a, c)
    assert torch.equal(st_w, st_n)
    return no_ws, nat.decode_stats(st_n.cpu().numpy())


def test_noalloc_matches_workspace_entry_point_twice(ref, nat):
    big = [I.config("m4n256")["problem"],
           I.make_problem(3, 100, 5, 7, nu_min=-1.3, nu_max=0.7, p=6.0, tau_lo=-40, tau_hi=30)]
    print("[gpu] noalloc: first call (M=4 N=256 F=129 + M=3 N=100 F=7, soft)", flush=True)
    zs = [I.logits(p["M"], p["N"], p["L"], 300 + i) for i, p in enumerate(big)]
    hs = [I.complex_gaussian(p["M"], p["N"], 310 + i) for i, p in enumerate(big)]
    z = torch.cat([torch.as_tensor(a).reshape(-1) for a in zs]).cuda()
    h = torch.cat([torch.as_tensor(a).reshape(-1) for a in hs]).cuda()
    (gz, gh, gs), sts = _both(nat, big, z, h, nat.WAVE_SOFT)
    ow = oz = 0
    for i, p in enumerate(big):
        M, N, L = p["M"], p["N"], p["L"]
        sr = ref.soft_waveform(zs[i].astype(np.float64), p["temperature"])
        st_ref, gs_ref, gh_ref = ref.evaluate(sr, hs[i].astype(np.complex128), p)
        assert abs(sts[i]["loss"] - st_ref["loss"]) <= 1e-4 * st_ref["loss"]
        assert _rel(gs[ow: ow + M * N].cpu().numpy(), gs_ref) <= 1e-4
        assert _rel(gh[ow: ow + M * N].cpu().numpy(), gh_ref) <= 1e-4
        gz_ref = ref.logit_grad(zs[i].astype(np.float64), p["temperature"], gs_ref)
        assert _rel(gz[oz: oz + M * N * L].cpu().numpy(), gz_ref) <= 1e-4
        ow += M * N
        oz += M * N * L
    print("[gpu] noalloc: second call (M=2 N=64 F=33, given waveforms, filter gradient only)", flush=True)
    small = [I.config("m2n64")["problem"]]
    p = small[0]
    s2 = torch.as_tensor(I.unimodular(p["M"], p["N"], 320)).reshape(-1).cuda()
    h2 = torch.as_tensor(I.complex_gaussian(p["M"], p["N"], 321)).reshape(-1).cuda()
    (gz2, gh2, gs2), sts2 = _both(nat, small, None, h2, nat.WAVE_GIVEN, s=s2, want_z=False, want_s=False)
    assert gz2 is None and gs2 is None
    st_ref, _, gh_ref = ref.evaluate(s2.cpu().numpy().reshape(2, 64).astype(np.complex128),
                                     h2.cpu().numpy().reshape(2, 64).astype(np.complex128), p)
    assert abs(sts2[0]["loss"] - st_ref["loss"]) <= 1e-4 * st_ref["loss"]
    assert _rel(gh2.cpu().numpy(), gh_ref) <= 1e-4

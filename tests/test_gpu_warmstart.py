"""The warm-start pipeline end to end at a small size: converged-run data from
paired starts, training on the MFMA network, time to target against random
starts (mechanics and invariants; the measured A/B at the M=4 N=512 size is
produced by `python -m paper_2604_25728_amd.warmstart`)."""
import numpy as np
import pytest

from paper_2604_25728_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def WS():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_25728_amd import native, warmstart
    native.load()
    return warmstart


def test_paired_logits_peak_at_the_noise_quantile(WS):
    eps = np.array([[-3.0, 0.0, 0.3]])
    z = WS.paired_logits(eps, 8)
    assert z.shape == (1, 3, 8)
    assert np.argmax(z[0, 1]) == 4  # Phi(0) = 1/2 -> level L/2
    assert np.allclose(z.max(axis=-1), np.cos(2 * np.pi * np.min(np.abs(
        np.arange(8)[None, :] / 8 - np.array([[0.0013499], [0.5], [0.6179114]])), axis=-1)), atol=1e-3)


def test_pipeline_small(WS):
    prob = I.make_problem(4, 64, 4, 9, p=8.0, w_psl=0.1, w_snrl=0.9, snrl_target_db=0.3)
    opt = I.make_opt(total_iters=40, T0=1.0, T1=0.2)
    print("[gpu] warm-start pipeline small", flush=True)
    data = WS.generate(prob, opt, range(500, 508), batch=4, iters=40)
    assert data["idx"].shape == (8, 4, 64) and data["idx"].max() < 4
    net, hist = WS.train(prob, data, epochs=3, batch=4, lr=3e-3)
    assert len(hist) == 3 and all(np.isfinite(hist))
    res = WS.time_to_target(prob, opt, net.params, range(4), iters=40, check_every=10, timed_seeds=2)
    assert res["seeds"] == 4 and 0.0 <= res["fraction_reached"] <= 1.0
    for p in res["per_seed"]:
        # a random run that ends within the SNRL bound reaches its own final PSL by the last checkpoint
        if p["random_final_snrl_db"] <= 0.5:
            assert p["random_iters"] is not None and p["random_iters"] <= 40
        else:
            assert p["random_iters"] is None
        assert p["warm_iters"] is None or p["warm_iters"] <= 40
    for t in res.get("timed_per_seed", []):
        assert t["random_s"] is None or t["random_s"] > 0


def test_trained_network_reaches_the_random_start_target_sooner(WS):
    """What the trained network gains over the method without it, at the size it
    was trained for (M=4 N=512 L=8 F=129, the paper's weighting eps = 0.1,
    2000 iterations): on 32 held-out seeds the random starts end within the
    0.5 dB SNRL bound, and the warm start reaches the random start's final
    hard PSL with its SNRL within 0.5 dB on most seeds, in far fewer
    iterations; a few seeds are also timed one design at a time."""
    cfg = I.config(WS.WORKLOAD)
    prob, opt = cfg["problem"], cfg["opt"]
    params = torch.tensor(WS.trained_params(), device="cuda")
    print("[gpu] warm start A/B on 32 held-out seeds", flush=True)
    res = WS.time_to_target(prob, opt, params, range(32), iters=opt["total_iters"], check_every=50, timed_seeds=4)
    print({k: v for k, v in res.items() if k not in ("per_seed", "timed_per_seed")})
    assert res["snrl_bound_db"] == 0.5
    assert res["random_within_bound"] >= 0.9
    assert res["fraction_reached"] >= 0.9
    assert res["median_ratio_iters"] <= 0.5
    assert res["median_warm_final_psl_db"] <= res["median_target_psl_db"]
    assert res["timed_warm_reached"] >= 0.75

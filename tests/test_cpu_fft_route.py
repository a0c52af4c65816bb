"""The CPU FFT-route baseline of bench.py (the paper's eq. 33-36 in numpy,
complex128) computes what the oracle's direct sums compute."""
import numpy as np

from paper_2604_25728_amd import inputs as I


def test_fft_route_matches_oracle(ref):
    import bench
    for prob in (I.make_problem(2, 24, 4, 5, nu_min=-0.7, nu_max=0.4, p=8.0, tau_lo=-20, tau_hi=15, w_snrl=0.6),
                 I.make_problem(3, 40, 4, 3, p=16.0)):
        rng = np.random.default_rng(3)
        s = np.exp(2j * np.pi * rng.random((prob["M"], prob["N"])))
        h = rng.standard_normal((prob["M"], prob["N"])) + 1j * rng.standard_normal((prob["M"], prob["N"]))
        loss, gs, gh = bench.fft_route_eval(s, h, prob)
        st, gs_ref, gh_ref = ref.evaluate(s, h, prob)
        assert abs(loss - st["loss"]) <= 1e-12 * st["loss"]
        assert np.abs(gs - gs_ref).max() <= 1e-10 * np.abs(gs_ref).max()
        assert np.abs(gh - gh_ref).max() <= 1e-10 * np.abs(gh_ref).max()

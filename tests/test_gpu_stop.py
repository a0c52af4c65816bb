"""The stopping criterion of Algorithm 1 on the device (sqngd_stop_update and
the stop mask of sqngd_set_stop_mask) against the host rule optim.StopRule:
the same decisions on the same checkpoint statistics, and a device-driven run
that equals, bit for bit, a run whose decisions the host takes."""
import numpy as np
import pytest

from paper_2604_25728_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_25728_amd import native, optim
    native.load()
    return native, optim


def test_stop_update_matches_stoprule(mods):
    nat, optim = mods
    print("[gpu] stop update vs StopRule", flush=True)
    n, checks, patience, gain = 7, 12, 3, 0.125   # gains exact in FP32 and FP64
    rng = np.random.default_rng(70)
    w = -20.0 - np.cumsum(rng.choice([0.0, 0.0625, 0.375], size=(checks, n)), axis=0)   # flat, slow, improving
    w[:, 6] = -20.0 - 0.375 * np.arange(checks)   # improving at every checkpoint: never stops
    w[4, 2] = np.nan                       # a non-finite checkpoint counts as a stall
    w[6:, 5] = w[5, 5] - gain              # exactly min_gain below the best: a stall
    best = torch.full((n,), float("inf"), device="cuda")
    stall = torch.zeros(n, dtype=torch.int32, device="cuda")
    stopped = torch.zeros(n, dtype=torch.int32, device="cuda")
    stop_iter = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    counter = torch.zeros(1, dtype=torch.int32, device="cuda")
    rule = optim.StopRule(n, patience, gain)
    want_iter = np.full(n, -1)
    for c in range(checks):
        words = np.zeros((n, nat.STATS_WORDS), dtype=np.int32)
        words.view(np.float32)[:, nat.STATS_FIELDS.index("pslr_db")] = w[c].astype(np.float32)
        counter.fill_(10 * (c + 1))
        nat.stop_update(torch.as_tensor(words).cuda(), gain, patience, counter, best, stall, stopped, stop_iter)
        ids = [i for i in range(n) if not rule.stopped[i]]
        for i in rule.update(ids, [float(np.float32(w[c, i])) for i in ids]):
            want_iter[i] = 10 * (c + 1)
    torch.cuda.synchronize()
    assert np.array_equal(stopped.cpu().numpy().astype(bool), rule.stopped)
    assert np.array_equal(stop_iter.cpu().numpy(), want_iter)
    assert np.array_equal(stall.cpu().numpy(), rule.stall)
    assert rule.stopped.any() and not rule.stopped.all()


def test_device_rule_matches_host_decisions(mods):
    """Six M=2 N=64 designs, checkpoints every 10 outer iterations, patience 2,
    0.25 dB minimum gain: the device-driven run (one graph per checkpoint)
    against a run of the same batch whose stop mask the host sets from
    StopRule after every checkpoint. Stop iterations and final states agree
    bit for bit; a stopped design's state is the one it had when it stopped."""
    nat, optim = mods
    print("[gpu] device stopping rule vs host decisions", flush=True)
    c = I.config("m2n64")
    probs, opt = [c["problem"]] * 6, dict(c["opt"], total_iters=200)
    seeds = list(range(40, 46))
    out = optim.optimise_on_device(probs, opt, seeds=seeds, max_iters=200, check_every=10, patience=2,
                                   min_gain_db=0.25, poll_every=1)
    ref = optim.SQNGD(probs, opt, seeds=seeds)
    mask = torch.zeros(6, dtype=torch.int32, device="cuda")
    ref.batch.set_stop_mask(mask)
    rule = optim.StopRule(6, 2, 0.25)
    stop_at = np.full(6, 200)
    snap = {}
    it = 0
    while it < 200 and not rule.stopped.all():
        ref.step(10)
        it += 10
        sts = ref.hard_stats()
        ids = [i for i in range(6) if not rule.stopped[i]]
        for i in rule.update(ids, [sts[i]["pslr_db"] for i in ids]):
            stop_at[i] = it
            mask[i] = 1
            snap[i] = ref.batch.unpack_z(ref.z, i).clone()
    torch.cuda.synchronize()
    got = np.array([d["stop_iter"] for d in out["designs"]])
    assert np.array_equal(got, stop_at), (got, stop_at)
    assert rule.stopped.any()
    for i in range(6):
        assert np.array_equal(out["designs"][i]["z"], ref.batch.unpack_z(ref.z, i).cpu().numpy()), i
        assert np.array_equal(out["designs"][i]["h"], ref.batch.unpack_w(ref.h, i).cpu().numpy()), i
        if i in snap:
            assert torch.equal(snap[i], ref.batch.unpack_z(ref.z, i))

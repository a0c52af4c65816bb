"""Host logic of the optimiser driver that needs no GPU: the stopping rule of
Algorithm 1 as read in optim.StopRule."""
import numpy as np
import pytest

from paper_2604_25728_amd.optim import StopRule


def test_first_checkpoint_never_stops():
    r = StopRule(2, patience=1)
    assert r.update([0, 1], [-5.0, np.inf]) == [1]  # a non-finite first WPSL is no improvement
    assert list(r.best) == [-5.0, np.inf]


def test_stall_counter_resets_on_improvement():
    r = StopRule(1, patience=3)
    seq = [-10.0, -10.0, -9.0, -10.5, -10.5, -10.5, -10.4]
    stops = [r.update([0], [w]) for w in seq]
    # improvements at -10.0 and -10.5; stalls after -10.5 reach 3 at the last value
    assert stops == [[], [], [], [], [], [], [0]]
    assert r.best[0] == -10.5 and r.stopped[0]


def test_min_gain_counts_small_improvements_as_stalls():
    r = StopRule(1, patience=2, min_gain_db=0.5)
    assert r.update([0], [-10.0]) == []
    assert r.update([0], [-10.4]) == []      # 0.4 dB < 0.5 dB: first stall, best unchanged
    assert r.best[0] == -10.0
    assert r.update([0], [-10.6]) == []      # 0.6 dB: improvement, counter reset
    assert r.update([0], [-10.7]) == []
    assert r.update([0], [-11.0]) == [0]


def test_designs_are_independent_and_ids_are_global():
    r = StopRule(4, patience=1)
    assert r.update([0, 1, 2, 3], [-1.0, -2.0, -3.0, -4.0]) == []
    assert r.update([0, 1, 2, 3], [-1.5, -2.0, -3.5, -3.0]) == [1, 3]
    assert r.update([0, 2], [-1.4, -3.6]) == [0]
    with pytest.raises(ValueError):
        r.update([1], [-9.0])                 # a stopped design takes no further checkpoints
    with pytest.raises(ValueError):
        StopRule(1, patience=0)


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    """No fallback: with libsqngd.so absent the binding raises instead of
    computing anything another way."""
    from paper_2604_25728_amd import native
    monkeypatch.setattr(native, "LIB_PATH", str(tmp_path / "libsqngd.so"))
    monkeypatch.setattr(native, "_lib", None)
    with pytest.raises(native.SQNGDError, match="is missing"):
        native.load()

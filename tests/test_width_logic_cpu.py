"""Host logic of the width tuner and the learned model (no GPU): best-width
tie-break, group split, regret, static-width choice, feature layout."""
import numpy as np

from paper_2210_06438_amd import learned, tune


def _records():
    recs = []
    for n in (8, 16):
        for rate in (1e3, 1e4, 1e5):
            for w in tune.WIDTHS:
                # a bowl in log2(w) whose bottom moves with the rate
                opt = np.log2(rate) / 2 - 3
                p99 = 100.0 + 10.0 * (np.log2(w) - opt) ** 2 + n
                recs.append({"n": n, "nfields": 11, "rate": rate, "width": w, "p99_us": p99})
    return recs


def test_best_width_and_tie_break():
    recs = [{"n": 8, "nfields": 6, "rate": 1.0, "width": w, "p99_us": p}
            for w, p in ((1, 5.0), (2, 3.0), (4, 3.0), (8, 9.0))]
    assert tune.best_width(recs) == {(8, 6, 1.0): (2, 3.0)}


def test_split_is_by_group_and_disjoint():
    recs = _records()
    train, test = learned.split(recs, test_frac=0.34, seed=1)
    assert set(train).isdisjoint(test) and len(train) + len(test) == 6 and len(test) == 2


def test_regret_and_static_width():
    recs = _records()
    g = (8, 11, 1e4)
    best = tune.best_width([r for r in recs if (r["n"], r["nfields"], r["rate"]) == g])[g][0]
    assert learned.regret(recs, g, best) == 0.0
    assert learned.regret(recs, g, 512) > 0.0
    w = learned.best_static_width(recs, learned.groups(recs))
    assert w in tune.WIDTHS


def test_features():
    f = learned.features(8, 11, 1e4, 64)
    assert f.shape == (5,)
    assert np.allclose(f, [6.0, 0.5, 1.0, 4.0, np.log2(tune.task_bytes(8, 11))])


class _FakeModel:
    rate_range = (1e3, 1e5)

    def __init__(self, pick):
        self.pick = pick

    def choose(self, n, nfields, rate, widths):
        return self.pick

    def choose_mix(self, mix, nfields, rate, widths):
        return self.pick


def test_judged_width_runs_the_pick_once_and_falls_back_when_it_saturates():
    calls = []

    def measure(w):
        calls.append(w)
        # widths below 8 cannot keep up with the rate; 32 has the lowest p99
        return {"width": w, "rate": 1e4, "throughput": 1e4 if w >= 8 else 2e3,
                "p99_us": 50.0 + abs(np.log2(w) - 5.0)}
    j = learned.JudgedWidth(_FakeModel(64))
    assert j.choose(8, 11, 1e4, measure) == (64, 1, "model") and calls == [64]
    calls.clear()
    j = learned.JudgedWidth(_FakeModel(2))
    assert j.choose(8, 11, 1e4, measure) == (32, 1 + len(tune.WIDTHS), "fallback_saturated")
    assert calls == [2] + tune.WIDTHS
    calls.clear()
    assert j.choose(8, 11, 1e6, measure) == (32, len(tune.WIDTHS), "fallback_rate")
    assert calls == tune.WIDTHS
    assert j.choose(8, 11, 1e4, measure, mix={8: 0.5, 16: 0.5})[2] == "fallback_saturated"


def test_saturated_uses_the_drain_slack():
    r = lambda tput: {"rate": 1e6, "throughput": tput}
    assert not learned.saturated(r(1e6)) and not learned.saturated(r(0.92e6))
    assert learned.saturated(r(0.85e6))

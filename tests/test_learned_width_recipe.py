"""The learned-width recipe on the stored width sweep (width + timeout
policy), trained in FP64 by the reference perceptron on the CPU: on
held-out condition groups the cost model's argmin width has a lower p99
regret than the best single static width chosen on the training groups.
This pins the gain to the recipe and the measured data, independently of
the HIP kernels that train the same model on the GPU."""
import numpy as np

from oracle import mlp_oracle as M
from paper_2210_06438_amd import learned, tune


def _choose(records, train, test, epochs=2000, lr=1e-3):
    rows = learned.in_groups(records, train)
    X = learned.features([r["n"] for r in rows], [r["nfields"] for r in rows],
                         [r["rate"] for r in rows], [r["width"] for r in rows])
    y = learned.target(rows)
    xm, xs = X.mean(0), X.std(0) + 1e-12
    ym, ys = y.mean(), y.std() + 1e-12
    p = M.init(0)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    first = None
    for k in range(1, epochs + 1):
        loss, g = M.loss_and_grad(p, (X - xm) / xs, (y - ym) / ys)
        first = loss if first is None else first
        p, m, v = M.adam(p, g, m, v, k, lr=lr)
    assert loss < 0.05 * first
    out = {}
    for grp in test:
        W = np.array(tune.WIDTHS)
        Xg = learned.features(np.full(len(W), grp[0]), np.full(len(W), grp[1]),
                              np.full(len(W), grp[2]), W)
        pred = M.forward(p, (Xg - xm) / xs)[0]
        out[grp] = int(W[int(np.argmin(pred))])
    return out


def test_sweep_shape():
    for name in ("timeout", "idle"):
        recs = learned.load_sweep(name)
        assert len(recs) == len(tune.WIDTHS) * len(tune.EDGES) * len(tune.FIELDS) * len(tune.RATES)
        assert len(learned.groups(recs)) == 42
        assert all(r["p99_us"] > 0 for r in recs)


def test_recipe_beats_best_static_width():
    recs = learned.load_sweep("timeout")
    mlp, static = [], []
    for sp in (0, 1, 3):
        train, test = learned.split(recs, seed=sp)
        assert len(train) == 34 and len(test) == 8
        sw = learned.best_static_width(recs, train)
        pick = _choose(recs, train, test)
        mlp.append(np.mean([learned.regret(recs, g, pick[g]) for g in test]))
        static.append(np.mean([learned.regret(recs, g, sw) for g in test]))
    assert np.mean(mlp) < 0.5 * np.mean(static), (mlp, static)


def test_target_ranks_widths_past_saturation():
    """The learning target is log(min(p99, 2 ms)) where a width keeps up
    (throughput within the drain slack of the rate), and grows with the
    throughput deficit where it does not, so two saturated widths with the
    same clipped p99 still differ by how far each falls behind."""
    rec = lambda p99, tput: {"p99_us": p99, "rate": 1e6, "throughput": tput}
    t = learned.target([rec(80.0, 0.99e6), rec(80.0, 0.95e6),
                        rec(5e6, 2e5), rec(9e6, 5e5), rec(1e3, 1e6)])
    assert t[0] == np.log(80.0) and t[1] == np.log(80.0)        # drain, not deficit
    assert np.isclose(t[2], np.log(2000.0) + np.log(5.0) - learned.DRAIN_SLACK)
    assert np.isclose(t[3], np.log(2000.0) + np.log(2.0) - learned.DRAIN_SLACK)
    assert t[2] > t[3] > np.log(2000.0) > t[4] == np.log(1e3)


def test_judged_recipe_beats_best_static_width_on_the_serving_sweep():
    """On the sweep of the current runtime with rates up to 2M tasks/s (the
    one the serving policy is trained on) the bare model's mean regret is
    dominated by picks that cannot keep up; with the exhaustive tuner as its
    judge (one run of the model's width, the full sweep only if that run
    falls behind the rate) both its mean and its median regret are below
    the best static width's, at far fewer runs than the sweep."""
    recs = learned.load_sweep("timeout_to2m")
    judged, static, runs = [], [], []
    for sp in (0, 1, 2, 3):
        train, test = learned.split(recs, seed=sp)
        sw = learned.best_static_width(recs, train)
        pick = _choose(recs, train, test)
        for g in test:
            meas = learned.sweep_measure(recs, g)
            w, n_runs = pick[g], 1
            if learned.saturated(meas(w)):
                w = tune.best_width([meas(x) for x in tune.WIDTHS])[g][0]
                n_runs += len(tune.WIDTHS)
            judged.append(learned.regret(recs, g, w))
            static.append(learned.regret(recs, g, sw))
            runs.append(n_runs)
    assert np.mean(judged) < np.mean(static), (np.mean(judged), np.mean(static))
    assert np.median(judged) < np.median(static), (np.median(judged), np.median(static))
    assert np.mean(runs) < len(tune.WIDTHS) / 2, np.mean(runs)

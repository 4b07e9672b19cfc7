"""Learned aggregation width: a 5-64-64-1 FP32 perceptron trained on the GPU
by the library's own kernels (hydro_mlp_forward / _mse / _backward / _adam)
on timings that the width sweeps produce, used to pick the width of a
serving condition without sweeping it.

Features of (n, nfields, rate, width): log2 width, n/16, nfields/11,
log10 rate, log2 bytes per task.  Target (target()): log p99 latency,
standardised, with p99 clipped at OVERLOAD_US first: above it the width
cannot keep up with the arrival rate, the queue grows for as long as the run
lasts, and the exact figure measures the run's length rather than the
width, while its magnitude (up to seconds) would otherwise dominate the
squared error; plus the throughput deficit log(rate / throughput), which
still ranks the widths that cannot keep up.
The chosen width of a condition is the argmin of the prediction over the
candidate widths.  The exhaustive tuner (tune.py) is its judge and fallback
(JudgedWidth): the model's width is run once, and only if that run falls
behind the offered rate -- the case in which a wrong width costs most, since
p99 then grows with the length of the run -- or the rate lies outside the
trained range is every candidate width run and the best one taken.

Sweeps stored under data/ (made by tune.py on one MI355X):
  width_sweep_timeout.json       launch on width or 50 us timeout only (420 records)
  width_sweep_idle.json          also launch whenever a stream is idle (420)
  width_sweep_idle_r3.json       the same, median p99 of 3 arrival sequences per point (420)
  width_sweep_timeout_to2m.json  width or timeout, the runtime with multi-class launches and
                                 amax partials, rates up to 2M tasks/s (600)
"""
from __future__ import annotations

import ctypes
import json
import math
import os

import numpy as np

from . import hydroagg
from .tune import WIDTHS, best_width, task_bytes

NPARAM = 4609
OVERLOAD_US = 2000.0
# shortfalls of the measured throughput below the offered rate up to this
# (log) fraction are the finite run's drain, not a width that cannot keep up
DRAIN_SLACK = 0.1


def target(records, overload_us=OVERLOAD_US):
    """Learning target of each record: log p99 with p99 clipped at
    overload_us, plus the throughput deficit log(rate / throughput) beyond
    DRAIN_SLACK.  Past saturation the clipped p99 is the same for every
    width; the deficit still ranks them (how far each falls behind the
    offered rate), and it is zero wherever the width keeps up."""
    p99 = np.array([r["p99_us"] for r in records], dtype=np.float64)
    rate = np.array([r["rate"] for r in records], dtype=np.float64)
    tput = np.array([r["throughput"] for r in records], dtype=np.float64)
    deficit = np.maximum(np.log(rate / np.maximum(tput, 1e-9)) - DRAIN_SLACK, 0.0)
    return np.log(np.minimum(p99, overload_us)) + deficit
DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


def load_sweep(name="timeout"):
    """Records of a stored width sweep ("timeout" or "idle")."""
    with open(os.path.join(DATA, f"width_sweep_{name}.json")) as f:
        return json.load(f)["records"]


def _setup(L):
    if getattr(L, "_mlp_ready", False):
        return L
    V = ctypes.c_void_p
    L.hydro_mlp_forward.argtypes = [V, V, ctypes.c_int32, V, V, V]
    L.hydro_mlp_backward.argtypes = [V, V, V, V, ctypes.c_int32, V, V, V]
    L.hydro_mlp_mse.argtypes = [V, V, ctypes.c_int32, V, V, V]
    L.hydro_mlp_adam.argtypes = [V, V, V, V, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, ctypes.c_float, ctypes.c_int32, V]
    for n in ("hydro_mlp_forward", "hydro_mlp_backward", "hydro_mlp_mse", "hydro_mlp_adam"):
        getattr(L, n).restype = ctypes.c_int
    L._mlp_ready = True
    return L


def _lib():
    return _setup(hydroagg.lib())


def _check(rc):
    if rc != 0:
        raise hydroagg.HydroError(rc, hydroagg.lib().hydro_last_error().decode())


def features(n, nfields, rate, width):
    n = np.asarray(n, dtype=np.float64)
    nf = np.asarray(nfields, dtype=np.float64)
    b = ((n + 6) ** 3 + n ** 3) * nf * 8
    return np.stack(np.broadcast_arrays(np.log2(np.asarray(width, dtype=np.float64)), n / 16.0,
                                        nf / 11.0, np.log10(np.asarray(rate, dtype=np.float64)),
                                        np.log2(b)), axis=-1)


def init_params(seed=0):
    """He-uniform weights, zero biases (flat layout W1 b1 W2 b2 W3 b3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for shape, fan in (((64, 5), 5), ((64,), 0), ((64, 64), 64), ((64,), 0), ((64,), 64), ((1,), 0)):
        if fan:
            lim = math.sqrt(6.0 / fan)
            parts.append(rng.uniform(-lim, lim, size=shape).ravel())
        else:
            parts.append(np.zeros(int(np.prod(shape))))
    return np.concatenate(parts).astype(np.float32)


class MLP:
    """Device-resident parameters and Adam state; every step runs in the
    library's HIP kernels on `stream` (torch tensors provide the memory)."""

    def __init__(self, params=None, seed=0, device="cuda:0"):
        import torch
        self.torch = torch
        self.dev = torch.device(device)
        p = init_params(seed) if params is None else np.asarray(params, dtype=np.float32)
        self.p = torch.from_numpy(p.copy()).to(self.dev)
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.g = torch.zeros_like(self.p)
        self.step_no = 0

    def _x(self, X):
        t = self.torch
        return t.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(self.dev)

    def forward(self, X, act=None):
        L = _lib()
        x = self._x(X) if isinstance(X, np.ndarray) else X
        rows = x.shape[0]
        y = self.torch.empty(rows, dtype=self.torch.float32, device=self.dev)
        _check(L.hydro_mlp_forward(self.p.data_ptr(), x.data_ptr(), rows, y.data_ptr(),
                                   act.data_ptr() if act is not None else None, None))
        return y

    def gradient(self, X, T):
        """(loss, grad) of the MSE on (X, T), on the device."""
        t = self.torch
        L = _lib()
        x = self._x(X) if isinstance(X, np.ndarray) else X
        tgt = t.from_numpy(np.ascontiguousarray(T, dtype=np.float32)).to(self.dev) \
            if isinstance(T, np.ndarray) else T
        rows = x.shape[0]
        act = t.empty(2 * rows * 64, dtype=t.float32, device=self.dev)
        scratch = t.empty_like(act)
        dy = t.empty(rows, dtype=t.float32, device=self.dev)
        loss = t.empty(1, dtype=t.float32, device=self.dev)
        y = self.forward(x, act)
        _check(L.hydro_mlp_mse(y.data_ptr(), tgt.data_ptr(), rows, dy.data_ptr(),
                               loss.data_ptr(), None))
        _check(L.hydro_mlp_backward(self.p.data_ptr(), x.data_ptr(), act.data_ptr(), dy.data_ptr(),
                                    rows, scratch.data_ptr(), self.g.data_ptr(), None))
        return loss, self.g

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step_no += 1
        _check(_lib().hydro_mlp_adam(self.p.data_ptr(), self.g.data_ptr(), self.m.data_ptr(),
                                     self.v.data_ptr(), NPARAM, lr, b1, b2, eps, self.step_no,
                                     None))

    def fit(self, X, T, epochs=2000, lr=1e-3):
        """Full-batch Adam on the MSE; returns the loss curve (every 100)."""
        x = self._x(X)
        tgt = self.torch.from_numpy(np.ascontiguousarray(T, dtype=np.float32)).to(self.dev)
        curve = []
        for e in range(epochs):
            loss, _ = self.gradient(x, tgt)
            self.adam(lr=lr)
            if e % 100 == 0 or e == epochs - 1:
                curve.append(float(loss.item()))
        return curve

    def predict(self, X):
        y = self.forward(X)
        return y.cpu().numpy().astype(np.float64)

    def params(self):
        return self.p.cpu().numpy()


# ---------------------------------------------------------------------------
def groups(records):
    return sorted({(r["n"], r["nfields"], r["rate"]) for r in records})


def split(records, test_frac=0.2, seed=5):
    """Split by condition group (never by row): (train groups, test groups)."""
    g = groups(records)
    rng = np.random.Generator(np.random.PCG64(seed))
    order = rng.permutation(len(g))
    ntest = max(1, int(round(test_frac * len(g))))
    test = sorted(g[i] for i in order[:ntest])
    train = sorted(g[i] for i in order[ntest:])
    return train, test


def saturated(record, slack=DRAIN_SLACK):
    """True when a serving run fell behind its offered rate: throughput
    deficit log(rate / throughput) beyond the drain slack."""
    return math.log(record["rate"] / max(record["throughput"], 1e-9)) > slack


class JudgedWidth:
    """The width model with the exhaustive tuner as its judge and fallback.

    choose(n, nfields, rate, measure) -> (width, runs, how).  measure(width)
    serves the condition at that width once and returns its record (p99_us,
    throughput, rate): a short serving run online, a lookup in a stored sweep
    offline.  The model's width is measured once (runs = 1); if the run is
    saturated (saturated()) every candidate width is measured and the lowest
    p99 taken (runs = 1 + len(widths), how = "fallback_saturated").  A rate
    outside the rates the model was trained on goes to the exhaustive tuner
    directly (runs = len(widths), how = "fallback_rate")."""

    def __init__(self, model, widths=WIDTHS):
        self.model = model
        self.widths = list(widths)

    def _exhaustive(self, measure):
        recs = [measure(w) for w in self.widths]
        best = min(recs, key=lambda r: (r["p99_us"], r["width"]))
        return int(best["width"]), len(recs)

    def choose(self, n, nfields, rate, measure, mix=None):
        lo, hi = self.model.rate_range
        if not lo <= rate <= hi:
            w, runs = self._exhaustive(measure)
            return w, runs, "fallback_rate"
        w = self.model.choose_mix(mix, nfields, rate, self.widths) if mix else \
            self.model.choose(n, nfields, rate, self.widths)
        if not saturated(measure(w)):
            return w, 1, "model"
        w, runs = self._exhaustive(measure)
        return w, runs + 1, "fallback_saturated"


class WidthModel:
    """Standardisation + MLP + argmin over candidate widths."""

    def __init__(self, seed=0, overload_us=OVERLOAD_US, device="cuda:0"):
        self.seed = seed
        self.overload_us = overload_us
        self.device = device
        self.mlp = None

    def fit(self, records, epochs=2000, lr=1e-3):
        X = features([r["n"] for r in records], [r["nfields"] for r in records],
                     [r["rate"] for r in records], [r["width"] for r in records])
        y = target(records, self.overload_us)
        rates = [r["rate"] for r in records]
        self.rate_range = (min(rates), max(rates))
        self.xm, self.xs = X.mean(0), X.std(0) + 1e-12
        self.ym, self.ys = y.mean(), y.std() + 1e-12
        self.mlp = MLP(seed=self.seed, device=self.device)
        self.curve = self.mlp.fit((X - self.xm) / self.xs, (y - self.ym) / self.ys,
                                  epochs=epochs, lr=lr)
        return self

    def predict_log_p99(self, n, nfields, rate, widths):
        X = features(np.full(len(widths), n), np.full(len(widths), nfields),
                     np.full(len(widths), rate), np.asarray(widths))
        return self.mlp.predict((X - self.xm) / self.xs) * self.ys + self.ym

    def choose(self, n, nfields, rate, widths=WIDTHS):
        pred = self.predict_log_p99(n, nfields, rate, widths)
        return int(widths[int(np.argmin(pred))])

    def choose_mix(self, mix, nfields, rate, widths=WIDTHS):
        """Width for a stream of mixed edges, mix = {n: fraction of tasks}:
        argmin of the mix-weighted predicted log p99."""
        pred = sum(f * self.predict_log_p99(n, nfields, rate, widths) for n, f in mix.items())
        return int(widths[int(np.argmin(pred))])


def regret(records, group, width):
    """(p99 at `width` - best p99) / best p99 for one condition group."""
    by = {r["width"]: r["p99_us"] for r in records
          if (r["n"], r["nfields"], r["rate"]) == group}
    best = min(by.values())
    return (by[width] - best) / best


def best_static_width(records, train_groups, widths=WIDTHS):
    """The single width with the lowest mean regret over the train groups."""
    scores = {w: np.mean([regret(records, g, w) for g in train_groups]) for w in widths}
    return min(scores, key=lambda w: (scores[w], w))


def in_groups(records, gs):
    gs = set(gs)
    return [r for r in records if (r["n"], r["nfields"], r["rate"]) in gs]


def sweep_measure(records, group):
    """measure(width) for JudgedWidth offline: the stored run of the group at
    that width (the measurement the tuner would make)."""
    by = {r["width"]: r for r in records if (r["n"], r["nfields"], r["rate"]) == group}
    return lambda w: by[w]


def evaluate(records, model, test_groups, static_width):
    rows = []
    judge = JudgedWidth(model)
    for g in test_groups:
        w = model.choose(*g)
        jw, runs, how = judge.choose(*g, measure=sweep_measure(records, g))
        best = best_width([r for r in records if (r["n"], r["nfields"], r["rate"]) == g])[g]
        rows.append({"group": list(g), "mlp_width": w, "best_width": best[0],
                     "mlp_regret": regret(records, g, w),
                     "judged_width": jw, "judged_regret": regret(records, g, jw),
                     "judged_runs": runs, "judged_how": how,
                     "static_regret": regret(records, g, static_width)})
    return {"static_width": static_width, "rows": rows,
            "mlp_mean_regret": float(np.mean([r["mlp_regret"] for r in rows])),
            "judged_mean_regret": float(np.mean([r["judged_regret"] for r in rows])),
            "static_mean_regret": float(np.mean([r["static_regret"] for r in rows])),
            "mlp_median_regret": float(np.median([r["mlp_regret"] for r in rows])),
            "judged_median_regret": float(np.median([r["judged_regret"] for r in rows])),
            "static_median_regret": float(np.median([r["static_regret"] for r in rows])),
            "exhaustive_runs_per_condition": len(WIDTHS), "mlp_runs_per_condition": 0,
            "judged_runs_per_condition": float(np.mean([r["judged_runs"] for r in rows]))}


def cross_validate(records, splits=range(10), epochs=2000, lr=1e-3, model_seed=0,
                   device="cuda:0"):
    """Train on the train groups of each split, pick widths for its held-out
    groups; mean regrets of the model and of the best static width."""
    out = []
    for sp in splits:
        train, test = split(records, seed=sp)
        static = best_static_width(records, train)
        m = WidthModel(seed=model_seed, device=device).fit(in_groups(records, train),
                                                           epochs=epochs, lr=lr)
        ev = evaluate(records, m, test, static)
        ev["split"] = sp
        ev["final_loss"] = m.curve[-1]
        out.append(ev)
    allrows = [r for e in out for r in e["rows"]]
    return {"splits": out,
            "mlp_mean_regret": float(np.mean([e["mlp_mean_regret"] for e in out])),
            "judged_mean_regret": float(np.mean([e["judged_mean_regret"] for e in out])),
            "static_mean_regret": float(np.mean([e["static_mean_regret"] for e in out])),
            "mlp_median_regret": float(np.median([r["mlp_regret"] for r in allrows])),
            "judged_median_regret": float(np.median([r["judged_regret"] for r in allrows])),
            "static_median_regret": float(np.median([r["static_regret"] for r in allrows])),
            "mlp_wins": int(sum(e["mlp_mean_regret"] < e["static_mean_regret"] for e in out)),
            "judged_wins": int(sum(e["judged_mean_regret"] < e["static_mean_regret"] for e in out)),
            "judged_runs_per_condition": float(np.mean([r["judged_runs"] for r in allrows])),
            "judged_fallbacks": int(sum(r["judged_how"] != "model" for r in allrows)),
            "conditions": len(allrows)}

"""The exhaustive width tuner on the GPU (tune.exhaustive: every candidate
width served on the same seeded arrival sequence, the lowest p99 kept) and
the learned width judged by it online: JudgedWidth measures the model's
width with a short serving run and falls back to the tuner's sweep when that
run falls behind the offered rate or the rate is outside the trained range."""
import numpy as np
import pytest

from paper_2210_06438_amd import learned, tune

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

WIDTHS = [1, 4, 16, 64]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return "cuda:0"


def test_exhaustive_tuner_keeps_the_lowest_p99(dev):
    w, recs = tune.exhaustive(8, 6, 20000.0, widths=WIDTHS, seconds=0.05, min_tasks=400)
    print("exhaustive:", [(r["width"], round(r["p99_us"], 1), round(r["throughput"])) for r in recs],
          "->", w, flush=True)
    assert [r["width"] for r in recs] == WIDTHS
    assert all(r["p99_us"] > 0 and r["throughput"] > 0 for r in recs)
    best = min(recs, key=lambda r: (r["p99_us"], r["width"]))
    assert w == best["width"]


def test_judged_width_online(dev):
    """A model trained on the stored sweep picks a width for a condition
    inside its range; the judge measures that width once.  A rate above the
    trained range goes straight to the tuner's sweep."""
    model = learned.WidthModel(device=dev).fit(learned.load_sweep("timeout_to2m"), epochs=400)
    pool = tune.Pool(8, 11, count=64)
    runs = []

    def measure_at(rate):
        def measure(w):
            rec = tune.run_condition(pool, rate, [w], seconds=0.02, min_tasks=400)[0]
            runs.append(w)
            return rec
        return measure
    w, n, how = learned.JudgedWidth(model, widths=WIDTHS).choose(8, 11, 20000.0, measure_at(20000.0))
    assert w in WIDTHS and how in ("model", "fallback_saturated")
    assert n == (1 if how == "model" else 1 + len(WIDTHS)) and len(runs) == n
    runs.clear()
    w, n, how = learned.JudgedWidth(model, widths=WIDTHS).choose(8, 11, 5e6, measure_at(5e6))
    assert how == "fallback_rate" and n == len(WIDTHS) and runs == WIDTHS and w in WIDTHS

"""The width cost model trained on the GPU by the library's HIP kernels on
the stored width sweep (width + timeout policy): over ten group splits its
picks on the held-out groups have a lower p99 regret than the best static
width chosen on each split's training groups, without any sweep of the
held-out conditions."""
import numpy as np
import pytest

from paper_2210_06438_amd import learned

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return "cuda:0"


def test_learned_width_beats_static(dev):
    recs = learned.load_sweep("timeout")
    cv = learned.cross_validate(recs, splits=range(10), device=dev)
    for e in cv["splits"]:
        print(f"split {e['split']}: static W {e['static_width']} regret "
              f"{e['static_mean_regret']:.3f}, model {e['mlp_mean_regret']:.3f}", flush=True)
        assert np.isfinite(e["final_loss"]) and e["final_loss"] < 0.1
    assert cv["mlp_mean_regret"] < 0.5 * cv["static_mean_regret"], cv
    assert cv["mlp_wins"] >= 7, cv


def test_judged_model_beats_static_on_the_serving_sweep(dev):
    """The sweep the serving policy is trained on (current runtime, rates up
    to 2M tasks/s): with the exhaustive tuner as judge and fallback the
    GPU-trained model's picks have a lower mean and median p99 regret than
    the best static width, on at least 7 of 10 splits, at fewer than half
    the runs of the exhaustive sweep per condition."""
    recs = learned.load_sweep("timeout_to2m")
    cv = learned.cross_validate(recs, splits=range(10), device=dev)
    print(f"judged: mean {cv['judged_mean_regret']:.3f} median {cv['judged_median_regret']:.3f} "
          f"wins {cv['judged_wins']}/10, {cv['judged_runs_per_condition']:.2f} runs per condition, "
          f"{cv['judged_fallbacks']} fallbacks of {cv['conditions']}; static mean "
          f"{cv['static_mean_regret']:.3f} median {cv['static_median_regret']:.3f}; bare model "
          f"mean {cv['mlp_mean_regret']:.3f}", flush=True)
    assert cv["judged_mean_regret"] < cv["static_mean_regret"], cv
    assert cv["judged_median_regret"] < cv["static_median_regret"], cv
    assert cv["judged_wins"] >= 7, cv
    assert cv["judged_runs_per_condition"] < len(learned.WIDTHS) / 2, cv


def test_choose_is_a_candidate_width(dev):
    recs = learned.load_sweep("timeout")
    m = learned.WidthModel(device=dev).fit(recs, epochs=200)
    for g in learned.groups(recs)[:5]:
        assert m.choose(*g) in learned.WIDTHS

"""Host side of the learned selector (Sec. III-D with the MLP that replaces
the paper's tree): the committed label set and model, the split and the
normalization, the regret report, and the held-out regret of the committed
model reproduced with the oracle's FP64 forward pass (no GPU)."""
import json
import math

import numpy as np
import pytest

import oracle
from paper_1711_05487_amd import learn

LABELS = learn.WEIGHTS.replace("mlp16_mi355x.json", "labels_mi355x.jsonl")


@pytest.fixture(scope="module")
def recs():
    return learn.read_labels(LABELS)


@pytest.fixture(scope="module")
def model():
    return learn.load_weights()


def unflatten(flat):
    out, k = [], 0
    for fi, fo in zip(learn.SIZES[:-1], learn.SIZES[1:]):
        out.append(np.asarray(flat[k:k + fo * fi], dtype=np.float64).reshape(fo, fi))
        k += fo * fi
        out.append(np.asarray(flat[k:k + fo], dtype=np.float64))
        k += fo
    assert k == len(flat)
    return out


def test_label_records_are_well_formed(recs):
    assert len(recs) == 2000
    assert [r["index"] for r in recs] == list(range(2000))
    for r in recs:
        t = np.array(r["times_ms"])
        assert len(r["features"]) == 16 and np.all(np.isfinite(r["features"]))
        assert t.shape == (learn.K,) and np.all(t > 0)
        # the label is the fastest variant, ties to the lower id
        assert r["label"] == int(np.argmin(t))


def test_split_is_by_seed_and_about_one_fifth(recs):
    tr, te = learn.split(recs)
    assert len(tr) + len(te) == len(recs)
    assert not ({r["seed"] for r in tr} & {r["seed"] for r in te})
    assert 0.17 < len(te) / len(recs) < 0.23
    tr2, te2 = learn.split(list(reversed(recs)))
    assert sorted(r["seed"] for r in te2) == sorted(r["seed"] for r in te)


def test_normalization_is_log_mean_and_population_sd(recs):
    mu, sd = learn.normalization(recs[:50])
    F = np.array([[math.log2(1.0 + v) for v in r["features"]] for r in recs[:50]])
    for j in range(16):
        col = F[:, j]
        m = sum(col) / len(col)
        s = math.sqrt(sum((c - m) ** 2 for c in col) / len(col))
        assert mu[j] == pytest.approx(m, rel=1e-12, abs=1e-12)
        assert sd[j] == pytest.approx(s if s >= 1e-6 else 1.0, rel=1e-9, abs=1e-12)


def test_regret_report_by_hand():
    recs = [{"times_ms": [2.0, 1.0, 4.0], "profile_ms": 2.0},
            {"times_ms": [3.0, 6.0, 1.5], "profile_ms": 3.0}]
    rep = learn.evaluate(recs, np.array([1, 0]))
    # selected/best: 1 and 2 -> geomean sqrt(2); plain/best: 2 and 2
    assert rep["geomean_sel_over_best"] == pytest.approx(math.sqrt(2.0))
    assert rep["geomean_plain_over_best"] == pytest.approx(2.0)
    assert rep["geomean_profile_over_best"] == pytest.approx(2.0)
    assert rep["geomean_speedup_vs_plain"] == pytest.approx(math.sqrt(2.0))
    assert rep["accuracy"] == 0.5


def test_committed_model_within_ten_percent_on_held_out(recs, model):
    """The committed weights, run through the oracle's FP64 forward pass on the
    held-out fifth: geometric mean of t_selected / t_best at most 1.10 (the
    GPU's FP32 forward reports 1.017 at training time)."""
    params, mu, sd, meta = model
    assert len(params) == 6288 and np.all(sd > 0) and np.all(np.isfinite(mu))
    _, te = learn.split(recs)
    X = oracle.normalize(np.array([r["features"] for r in te]), mu, sd)
    logits, _ = oracle.mlp_forward(unflatten(params), X)
    rep = learn.evaluate(te, np.argmax(logits, axis=1))
    assert rep["n"] == meta["test"]["n"]
    assert rep["geomean_sel_over_best"] <= 1.10
    assert rep["geomean_sel_over_best"] == pytest.approx(meta["test"]["geomean_sel_over_best"],
                                                         rel=0.01)


BOUNDS = learn.WEIGHTS.replace("mlp16_mi355x.json", "bounds_mi355x.jsonl")


def test_profile_thresholds_are_the_grid_search_optimum():
    """The library's default thresholds and class -> remedy map are what a
    grid search (Sec. III-C) over the committed MI355X bounds records picks
    on the training split; on the held-out split they beat the paper's KNC
    thresholds with either map. Runs the library's own rule (host code)."""
    recs = learn.read_labels(BOUNDS)
    assert len(recs) == 400
    for r in recs:
        assert len(r["bounds"]) == 6 and len(r["catalogue_ms"]) == 16
        assert r["set_times_ms"]["0"] > 0
    tr, te = learn.split(recs)
    d = learn.default_thresholds()
    grid = dict(grid_ml=[1.0, 1.25, 1.5, 2.0], grid_imb=[1.0, 1.24, 1.5, 2.0],
                grid_mb=[0.5, 0.8, 1.0])
    best, g_best, g_paper = learn.tune_thresholds(tr, 1, defaults=learn.PAPER_THRESHOLDS, **grid)
    assert best == d and g_best > g_paper
    held = learn.profile_regret(te, d, 1)
    assert held[0] < 1.1
    assert held[0] < learn.profile_regret(te, learn.PAPER_THRESHOLDS, 0)[0]
    assert held[0] < learn.profile_regret(te, learn.PAPER_THRESHOLDS, 1)[0]


def test_set_time_resolves_equivalent_sets():
    r = {"set_times_ms": {"0": 2.0, "8": 1.0}, "catalogue_ms": list(range(1, 17))}
    assert learn.set_time(r, 8) == 1.0
    assert learn.set_time(r, 8 | 4) == 1.0          # the merge path wins over decomposition
    cat = learn.catalogue()
    assert learn.set_time(r, 9) == r["catalogue_ms"][cat.index(9)]

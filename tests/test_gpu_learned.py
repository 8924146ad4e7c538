"""The trained learned selector against the timings that label it, on GPU:
regret against the exhaustive timings on the held-out split (within 10% of the
best variant), the gain over the method without the network (plain CSR and
the profile-guided selector), and the selection cost against one plain
SpMV. The labels and weights are the committed training set and model
(`paper_1711_05487_amd/weights/`, written by `python -m
paper_1711_05487_amd.learn`)."""
import os

import numpy as np
import pytest
import torch

import paper_1711_05487_amd as pkg
from paper_1711_05487_amd import learn
from spmv_cases import check_f64, matrix, xvec

pytestmark = pytest.mark.gpu

LABELS = os.path.join(os.path.dirname(learn.WEIGHTS), "labels_mi355x.jsonl")


def held_out():
    recs = learn.read_labels(LABELS)
    _, te = learn.split(recs)
    return te


def test_regret_within_ten_percent_on_held_out():
    params, mu, sd, meta = learn.load_weights()
    te = held_out()
    assert len(te) >= 300
    pred = learn.predict(params, mu, sd, [r["features"] for r in te])
    ev = learn.evaluate(te, pred)
    print(ev)
    assert ev["geomean_sel_over_best"] <= 1.10
    # the network gains over the method without it: plain CSR, and the
    # profile-guided classifier of Sec. III-C
    assert ev["geomean_speedup_vs_plain"] > 1.2
    assert ev["geomean_sel_over_best"] < ev["geomean_profile_over_best"]


def test_training_reproduces_committed_model():
    # retraining with the same seeds reproduces the committed weights bit for bit
    recs = learn.read_labels(LABELS)
    tr, _ = learn.split(recs)
    params, mu, sd, _ = learn.train(tr, epochs=learn.load_weights()[3].get("epochs", 200))
    p0, mu0, sd0, _ = learn.load_weights()
    assert np.array_equal(params, p0)
    assert np.array_equal(mu, mu0) and np.array_equal(sd, sd0)


@pytest.mark.parametrize("name", ["st27_128", "unif20", "rmat22"])
def test_learned_selection_cost_below_one_plain_spmv(name):
    """Features + inference + decision (t_select_ms, the median of five
    selections) below one plain SpMV on the configurations with NNZ >= 10^6."""
    learn.install()
    n, m, rp, col, val = matrix(name)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    x = torch.from_numpy(xvec(name, m)).cuda()
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    A.select("plain")
    A.spmv(x, y)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(20):
        A.spmv(x, y)
    e1.record(s)
    e1.synchronize()
    t_plain = e0.elapsed_time(e1) / 20
    costs = []
    for _ in range(5):
        info = A.select("learned")
        assert info["fallback"] == 0
        costs.append(info["t_select_ms"])
    print(name, "t_select_ms", costs, "t_plain_ms", t_plain, "variant", info["variant_id"])
    assert float(np.median(costs)) < t_plain
    y = A.spmv(x)
    torch.cuda.synchronize()
    check_f64(y.cpu().numpy(), rp, col, val, x.cpu().numpy(), f"learned {name}")
    A.close()


def test_learned_selection_parity_on_config_matrices():
    learn.install()
    for name in ("lap100", "rmat14", "unif14", "st27_24"):
        n, m, rp, col, val = matrix(name)
        A = pkg.CsrMatrix(rp, col, val)
        info = A.select("learned")
        assert info["fallback"] == 0 and 0 <= info["variant_id"] < 16
        x = xvec(name, m)
        y = A.spmv(torch.from_numpy(x).cuda())
        torch.cuda.synchronize()
        check_f64(y.cpu().numpy(), rp, col, val, x, f"learned {name}")


def test_regret_same_session_on_held_out_sample():
    """The regret judge re-timed now (the profiling selector's exhaustive
    timing as the reference, Sec. IV-D): on 24 held-out matrices of the suite
    (N <= 2^20, to keep generation short), the learned plan and all 16
    catalogue variants are timed in this session with the same protocol,
    and the geometric mean of t_learned / t_best stays within 10%."""
    import synth
    learn.install()
    te = [r for r in held_out() if r["n"] <= (1 << 20)]
    te = te[:: max(1, len(te) // 24)][:24]
    ratios = []
    for r in te:
        name, (n, m, rp, col, val) = synth.suite_matrix(r["index"])
        A = pkg.CsrMatrix(rp, col, val, n_cols=m)
        x = torch.ones(m, dtype=torch.float64, device="cuda")
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        times = learn.time_variants(A, x, y, calls=32, runs=3)
        info = A.select("learned")
        assert info["fallback"] == 0
        A.spmv(x, y)
        t_sel = learn._time_current(A, x, y, 32, 3)
        ratios.append(t_sel / min(times))
        A.close()
    gm = float(np.exp(np.mean(np.log(ratios))))
    print("same-session t_learned / t_best:", gm, "p90", float(np.percentile(ratios, 90)), len(ratios))
    assert gm <= 1.10


def test_features_outside_the_training_range_fall_back_to_profile():
    """The learned path's range test: the largest |standardized feature| is
    reported, equal to the oracle's normalization of the same features with
    the model's mu and sigma; past ood_z the profile-guided rule decides;
    ood_z = 0 turns the test off; a 1 x 1 matrix lies outside the range of
    the training suite at the default bound; invalid bounds are refused."""
    import oracle
    learn.install()
    _, mu, sd, _ = learn.load_weights()
    n, m, rp, col, val = matrix("st27_24")
    x = xvec("st27_24", m)
    A = pkg.CsrMatrix(rp, col, val)
    f, _, _ = A.inspect()
    z = float(np.abs(oracle.normalize(f, np.asarray(mu), np.asarray(sd))).max())
    assert 0.0 < z < 4.0
    info = A.select("learned")
    assert info["fallback"] == 0 and info["feature_z_max"] == pytest.approx(z, rel=1e-12)
    info = A.select("learned", ood_z=0.5 * z)
    assert info["fallback"] == 1 and info["classes"] >= 0  # the profile rule ran
    assert info["feature_z_max"] == pytest.approx(z, rel=1e-12)
    y = A.spmv(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    check_f64(y.cpu().numpy(), rp, col, val, x, "out-of-range fallback plan")
    assert A.select("learned", ood_z=0.0)["fallback"] == 0
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(pkg.CsrError):
            A.select("learned", ood_z=bad)
    assert A.select("profile")["feature_z_max"] == 0.0
    A.close()
    T = pkg.CsrMatrix(np.array([0, 1], dtype=np.int32), np.array([0], dtype=np.int32),
                      np.array([2.0]), n_cols=1)
    info = T.select("learned")
    assert info["fallback"] == 1 and info["feature_z_max"] > 4.0
    y = T.spmv(torch.tensor([0.5], dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    assert y.item() == 1.0
    T.close()

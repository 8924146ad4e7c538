"""Pins of the oracle's selection logic: the per-class bounds (Sec. III-B)
with hand-computed numbers, the profile-guided rule (Sec. III-C, Fig. 4) as a
truth table, the class -> optimization map (Sec. III-E, Table II), the
amortization count (Sec. IV-D, Eq. (2)) and the FP64 MLP against central
finite differences and torch autograd / torch.optim.Adam (library routines)."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth


def test_bounds_hand_computed():
    # 1e6 nonzeros, 1e5 rows, FP64/int32: S_CSR = 12e6 + 4(1e5+1) B,
    # S_x = S_y = 8e5 B, B = 1e12 B/s.
    nnz, n = 1_000_000, 100_000
    s_fmt = oracle.format_bytes(n, n, nnz)
    assert s_fmt == 12_000_000 + 400_004
    pmb = oracle.p_mb(nnz, s_fmt, 8 * n, 8 * n, 1e12)
    assert math.isclose(pmb, 2e6 / (14_000_004 / 1e12), rel_tol=1e-15)
    ppk = oracle.p_peak(nnz, 8 * nnz, 8 * n, 8 * n, 1e12)
    assert math.isclose(ppk, 2e6 / (9_600_000 / 1e12), rel_tol=1e-15)
    assert ppk > pmb
    assert oracle.p_imb(nnz, [3.0, 1.0, 2.0]) == 2e6 / 2.0
    assert oracle.p_imb(nnz, [4.0, 1.0, 2.0, 3.0]) == 2e6 / 2.5
    assert oracle.b_for_footprint(100, 5e12, 10e12) == 10e12
    assert oracle.b_for_footprint(300 << 20, 5e12, 10e12) == 5e12


def test_classify_truth_table():
    C = oracle
    base = dict(p_csr=100.0, p_mb_=200.0, p_ml=100.0, p_imb_=100.0, p_cmp=300.0, p_peak_=400.0)
    assert C.classify(**base) == 0
    assert C.classify(**{**base, "p_imb_": 124.1}) == C.CLS_IMB
    assert C.classify(**{**base, "p_imb_": 124.0}) == 0          # strict >
    assert C.classify(**{**base, "p_ml": 125.1}) == C.CLS_ML
    assert C.classify(**{**base, "p_ml": 125.0}) == 0
    mb = {**base, "p_csr": 180.0, "p_ml": 180.0, "p_imb_": 180.0}
    assert C.classify(**mb) == C.CLS_MB                          # 180 >= 0.8 * 200
    assert C.classify(**{**mb, "p_csr": 159.0, "p_ml": 159.0, "p_imb_": 159.0}) == 0
    assert C.classify(**{**mb, "p_cmp": 150.0}) == C.CLS_CMP     # P_MB > P_CMP
    assert C.classify(**{**mb, "p_cmp": 500.0}) == C.CLS_CMP     # P_CMP > P_peak
    assert C.classify(**{**base, "p_imb_": 200.0, "p_ml": 200.0, "p_cmp": 150.0}) == (
        C.CLS_IMB | C.CLS_ML | C.CLS_CMP)
    # MB and CMP are mutually exclusive by construction
    for pc in np.linspace(50, 600, 23):
        c = C.classify(**{**mb, "p_cmp": float(pc)})
        assert not (c & C.CLS_MB and c & C.CLS_CMP)


def test_remedies_table():
    C = oracle
    assert C.remedies(0, False) == 0
    assert C.remedies(C.CLS_MB, False) == C.OPT_DELTA
    assert C.remedies(C.CLS_ML, False) == C.OPT_PREFETCH
    assert C.remedies(C.CLS_IMB, True) == C.OPT_DECOMP
    assert C.remedies(C.CLS_IMB, False) == C.OPT_MERGE
    assert C.remedies(C.CLS_CMP, False) == C.OPT_UNROLL
    assert C.remedies(C.CLS_IMB | C.CLS_CMP | C.CLS_ML, True) == (
        C.OPT_DECOMP | C.OPT_UNROLL | C.OPT_PREFETCH)
    # the map for a GPU on which prefetching and unrolling do not pay
    assert C.remedies(C.CLS_MB, False, 1) == C.OPT_DELTA
    assert C.remedies(C.CLS_ML, False, 1) == C.OPT_MERGE | C.OPT_DELTA
    assert C.remedies(C.CLS_IMB, True, 1) == C.OPT_DECOMP
    assert C.remedies(C.CLS_IMB, False, 1) == C.OPT_MERGE | C.OPT_DELTA
    assert C.remedies(C.CLS_CMP, False, 1) == 0
    assert C.remedies(C.CLS_ML | C.CLS_CMP, True, 1) == C.OPT_MERGE | C.OPT_DELTA
    assert C.remedies(C.CLS_ML | C.CLS_IMB, True, 1) == C.OPT_MERGE | C.OPT_DELTA | C.OPT_DECOMP
    with pytest.raises(AssertionError):
        C.remedies(C.CLS_MB, False, 2)
    cat = C.catalogue()
    assert len(cat) == 16 and len(set(cat)) == 16 and cat[0] == 0
    assert all(bin(s).count("1") <= 2 for s in cat)
    assert sum(1 for s in cat if bin(s).count("1") == 1) == 5


def test_n_iters_min():
    assert oracle.n_iters_min(1.0, 0.010, 0.008) == pytest.approx(500.0)
    assert oracle.n_iters_min(1.0, 0.010, 0.010) == float("inf")
    assert oracle.harmonic_mean([1.0, 2.0, 4.0]) == pytest.approx(3 / 1.75)


def test_rel_error_report():
    r = oracle.rel_error_report(np.array([1.0, 2.0, 0.0]), np.array([1.0, 2.5, 0.0]),
                                np.array([1.0, 5.0, 0.0]))
    assert r["max"] == 0.1 and r["zero_rows_exact"]
    r = oracle.rel_error_report(np.array([0.0, 1e-300]), np.array([0.0, 0.0]), np.array([1.0, 0.0]))
    assert not r["zero_rows_exact"]


# ------------------------------------------------------------------ MLP

SIZES = [16, 64, 64, 16]


def _data(b=32, seed=3):
    X = synth.vector(b * 16, seed).reshape(b, 16)
    y = synth.uindex(seed + 1, 0, np.arange(b, dtype=np.uint64), 16)
    return X, y


def test_mlp_grad_finite_differences():
    params = synth.mlp_init_weights(SIZES, 701)
    params = [p + 0.01 * synth.vector(p.size, 40 + k).reshape(p.shape) for k, p in enumerate(params)]
    X, y = _data()
    _, grads = oracle.mlp_loss_grad(params, X, y)
    h = 1e-6
    for k, p in enumerate(params):
        flat = p.reshape(-1)
        idx = synth.uindex(50 + k, 0, np.arange(12, dtype=np.uint64), flat.size)
        for q in idx:
            old = flat[q]
            flat[q] = old + h
            lp, _ = oracle.mlp_loss_grad(params, X, y)
            flat[q] = old - h
            lm, _ = oracle.mlp_loss_grad(params, X, y)
            flat[q] = old
            fd = (lp - lm) / (2 * h)
            g = grads[k].reshape(-1)[q]
            assert abs(fd - g) <= 1e-6 * max(1.0, abs(g)) + 1e-8


def test_mlp_against_torch_autograd_and_adam():
    params = synth.mlp_init_weights(SIZES, 701)
    X, y = _data(64, 9)
    tp = [torch.tensor(p, dtype=torch.float64, requires_grad=True) for p in params]
    opt = torch.optim.Adam(tp, lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    Xt, yt = torch.tensor(X), torch.tensor(y)
    for t in range(1, 4):
        loss, grads = oracle.mlp_loss_grad(params, X, y)
        opt.zero_grad()
        h = Xt
        for l in range(3):
            h = h @ tp[2 * l].T + tp[2 * l + 1]
            if l < 2:
                h = torch.relu(h)
        tl = torch.nn.functional.cross_entropy(h, yt)
        tl.backward()
        assert abs(tl.item() - loss) <= 1e-12 * abs(loss)
        for g, p in zip(grads, tp):
            assert np.allclose(g, p.grad.numpy(), rtol=1e-10, atol=1e-13)
        opt.step()
        params, m, v = oracle.adam_step(params, grads, m, v, t)
        for a, p in zip(params, tp):
            assert np.allclose(a, p.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_mlp_overfits_small_set():
    params = synth.mlp_init_weights(SIZES, 701)
    X, y = _data(32, 11)
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    for t in range(1, 600):
        _, g = oracle.mlp_loss_grad(params, X, y)
        params, m, v = oracle.adam_step(params, g, m, v, t, lr=1e-2)
    logits, _ = oracle.mlp_forward(params, X)
    assert np.all(np.argmax(logits, 1) == y)


def test_normalize():
    f = np.array([[0.0, 1.0, 3.0]])
    out = oracle.normalize(f, np.array([0.0, 1.0, 1.0]), np.array([1.0, 1.0, 2.0]))
    assert out.tolist() == [[0.0, 0.0, 0.5]]

"""Pins of the two error scales every parity bar rests on, from facts that do
not come from the oracle itself:

* absax, the per-row |A||x| that scales the FP64 bar 1e-12 (|A||x|)_i:
  closed forms on the 5-point Laplacian, the identity, a permutation and a
  hand-worked row with mixed signs.
* reduced_precision_bound, the FP32/BF16 bar gamma_{n+1}(2^-24) (|A_q||x_q|)_i
  (Higham, Accuracy and Stability of Numerical Algorithms, Sec. 3.1: a sum of
  n rounded products in any order errs by at most gamma_n sum |a||x|, gamma_k
  = k u / (1 - k u)): hand-computed values on one-row cases, and a worst-case
  FP32 summation whose actual error reaches most of the bound, so that a
  bound loosened by any constant factor, or built on the BF16 unit roundoff
  instead of FP32's, fails.
* the comparison helpers themselves reject a planted error just above their
  bar and accept one just below it.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from spmv_cases import check_f64, check_reduced

U32 = 2.0 ** -24  # unit roundoff of FP32 accumulation


def one_row(vals):
    vals = np.asarray(vals, dtype=np.float64)
    n = vals.size
    rp = np.array([0, n], dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    return rp, col, vals


# ---------------------------------------------------------------- absax


def test_absax_laplacian_closed_form():
    # 5-point Laplacian on 100 x 100: |A| 1 = 4 + (number of grid neighbours):
    # 8 inside, 7 on an edge, 6 at a corner; x of random signs and |x| = 1
    # gives the same
    n, m, rp, col, val = synth.laplacian2d(100)
    sign = np.where(synth.vector(m, 5) < 0, -1.0, 1.0)
    ab = oracle.absax(rp, col, val, sign)
    g = ab.reshape(100, 100)
    assert np.all(g[1:-1, 1:-1] == 8.0)
    for edge in (g[0, 1:-1], g[-1, 1:-1], g[1:-1, 0], g[1:-1, -1]):
        assert np.all(edge == 7.0)
    assert [g[0, 0], g[0, -1], g[-1, 0], g[-1, -1]] == [6.0] * 4
    assert ab.sum() == 9604 * 8 + 392 * 7 + 4 * 6


def test_absax_identity_and_permutation():
    n = 1000
    x = synth.vector(n, 17)
    eye_rp = np.arange(n + 1, dtype=np.int32)
    ab = oracle.absax(eye_rp, np.arange(n, dtype=np.int32), -np.ones(n), x)
    assert np.array_equal(ab, np.abs(x))
    pi = synth.permutation(n, 23)
    ab = oracle.absax(eye_rp, pi.astype(np.int32), np.ones(n), x)
    assert np.array_equal(ab, np.abs(x[pi]))


def test_absax_hand_worked_rows():
    # row 0: |-2||-1.5| + |3||-0.25| = 3 + 0.75; row 1 empty; row 2:
    # |0.5||4| + |-0.125||-1.5| + |1||0| = 2 + 0.1875
    rp = np.array([0, 2, 2, 5], dtype=np.int32)
    col = np.array([0, 2, 1, 0, 3], dtype=np.int32)
    val = np.array([-2.0, 3.0, 0.5, -0.125, 1.0])
    x = np.array([-1.5, 4.0, -0.25, 0.0])
    assert list(oracle.absax(rp, col, val, x)) == [3.75, 0.0, 2.1875]


# ---------------------------------------------------------------- FP32/BF16 bound


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_reduced_bound_hand_computed(storage):
    # all-ones rows: |A_q||x_q| = n and the bound is n (n+1) u / (1 - (n+1) u)
    expect = {1: 2 * U32 / (1 - 2 * U32),
              7: 56 * U32 / (1 - 2.0 ** -21),
              1000: 1001000 * U32 / (1 - 1001 * U32)}
    for n, b in expect.items():
        rp, col, val = one_row(np.ones(n))
        yq, bound = oracle.reduced_precision_bound(rp, col, val, np.ones(n), storage)
        assert yq[0] == float(n)
        assert bound[0] == pytest.approx(b, rel=1e-15)


def test_reduced_bound_uses_stored_values_and_fp32_x():
    # BF16 keeps 8 significand bits: 1 + 2^-10 is stored as 1; FP32 x: 1 + 2^-30
    # is rounded to 1. The bound and reference are those of the stored row.
    n = 7
    rp, col, val = one_row(np.full(n, 1.0 + 2.0 ** -10))
    x = np.full(n, 1.0 + 2.0 ** -30)
    yq, bound = oracle.reduced_precision_bound(rp, col, val, x, "bf16")
    assert yq[0] == 7.0
    assert bound[0] == pytest.approx(56 * U32 / (1 - 2.0 ** -21), rel=1e-15)
    # FP32 keeps 1 + 2^-10 exactly
    yq, bound = oracle.reduced_precision_bound(rp, col, val, x, "f32")
    assert yq[0] == 7.0 * (1.0 + 2.0 ** -10)
    assert bound[0] == pytest.approx(56 * U32 / (1 - 2.0 ** -21) * (1.0 + 2.0 ** -10), rel=1e-15)


def fp32_sequential(vals, x):
    s = np.float32(0.0)
    for a, b in zip(np.asarray(vals, dtype=np.float32), np.asarray(x, dtype=np.float32)):
        s = np.float32(s + np.float32(a * b))
    return float(s)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("n,frac", [(7, 0.74), (1000, 0.99)])
def test_reduced_bound_reached_by_worst_case_sum(storage, n, frac):
    # 1 followed by n-1 terms of 2^-24: each 1 + 2^-24 is a tie that rounds to
    # even (1), so the FP32 sum stays 1 and errs by (n-1) 2^-24 while the
    # bound is about (n+1) 2^-24: the error reaches (n-1)/(n+1) of it. Both
    # terms are exact in BF16 and FP32.
    vals = np.r_[1.0, np.full(n - 1, U32)]
    x = np.ones(n)
    rp, col, val = one_row(vals)
    yq, bound = oracle.reduced_precision_bound(rp, col, val, x, storage)
    assert yq[0] == 1.0 + (n - 1) * U32
    got = fp32_sequential(vals, x)
    assert got == 1.0
    err = abs(got - yq[0])
    assert err == (n - 1) * U32
    assert err <= bound[0]
    assert err >= frac * bound[0]


def test_reduced_bound_single_product_rounding():
    # n = 1: only the product rounds. (1 + 2^-12)^2 = 1 + 2^-11 + 2^-24 is a
    # tie in FP32 and rounds to even, an error of exactly 2^-24 against a
    # bound of about 2^-23.
    a = 1.0 + 2.0 ** -12
    rp, col, val = one_row([a])
    yq, bound = oracle.reduced_precision_bound(rp, col, val, np.array([a]), "f32")
    got = fp32_sequential([a], [a])
    assert got == 1.0 + 2.0 ** -11
    err = abs(got - yq[0])
    assert err == U32
    assert 0.49 * bound[0] <= err <= bound[0]


# ---------------------------------------------------------------- the bars reject planted errors


def planted_case():
    n, m, rp, col, val = synth.stencil27(6)
    x = synth.vector(m, 31)
    return rp, col, val, x


def test_check_f64_rejects_planted_error():
    rp, col, val, x = planted_case()
    ref = oracle.spmv_accurate(rp, col, val, x)
    ab = oracle.absax(rp, col, val, x)
    i = 17
    ok = ref.copy()
    ok[i] += 0.99e-12 * ab[i]
    check_f64(ok, rp, col, val, x, "0.99 of the bar")
    bad = ref.copy()
    bad[i] += 1.01e-12 * ab[i]
    with pytest.raises(AssertionError, match=f"first row {i}"):
        check_f64(bad, rp, col, val, x, "1.01 of the bar")


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_check_reduced_rejects_planted_error(storage):
    rp, col, val, x = planted_case()
    yq, bound = oracle.reduced_precision_bound(rp, col, val, x, storage)
    i = 40
    ok = yq.copy()
    ok[i] -= 0.99 * bound[i]
    check_reduced(ok, rp, col, val, x, storage, "0.99 of the bound")
    bad = yq.copy()
    bad[i] -= 1.01 * bound[i]
    with pytest.raises(AssertionError, match=f"row {i}:"):
        check_reduced(bad, rp, col, val, x, storage, "1.01 of the bound")

"""Pins of the CPU oracle's SpMV (Sec. II, Fig. 2) against facts that do not
come from the oracle itself: identity and permutation matrices, the closed-form
row sums of the 2-D Laplacian, exact (dyadic) arithmetic where every summation
order agrees with numpy's dense product, brute force over every 0/1 pattern of
a 4x4 matrix, scipy's CSR product, and exact rational arithmetic."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth


def test_identity_is_bit_exact():
    n = 5000
    rp = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    x = synth.vector(n, 11)
    y = oracle.spmv(rp, col, np.ones(n), x)
    assert np.array_equal(y.view(np.uint64), x.view(np.uint64))


def test_permutation_is_bit_exact():
    n = 3001
    pi = synth.permutation(n, 12)
    assert np.array_equal(np.sort(pi), np.arange(n))
    rp = np.arange(n + 1, dtype=np.int32)
    x = synth.vector(n, 13)
    y = oracle.spmv(rp, pi.astype(np.int32), np.ones(n), x)
    assert np.array_equal(y, x[pi])


def test_laplacian_row_sums_closed_form():
    # A.1 for the 5-point Laplacian: 4 - (#neighbours) = 0 interior, 1 on an
    # edge, 2 at a corner; the total is 4*1 + ... = 2*4 + 1*392 = 400.
    n, _, rp, col, val = synth.laplacian2d(100)
    y = oracle.spmv(rp, col, val, np.ones(n))
    r, c = np.divmod(np.arange(n), 100)
    missing = (r == 0).astype(int) + (r == 99) + (c == 0) + (c == 99)
    assert np.array_equal(y, missing.astype(np.float64))
    assert y.sum() == 400.0


def test_empty_rows_give_positive_zero():
    rp = np.array([0, 0, 2, 2], dtype=np.int32)
    col = np.array([0, 1], dtype=np.int32)
    y = oracle.spmv(rp, col, np.array([1.0, -1.0]), np.array([1.0, 1.0]))
    assert y[0] == 0.0 and not np.signbit(y[0])
    assert y[2] == 0.0 and not np.signbit(y[2])
    assert y[1] == 0.0


@pytest.mark.parametrize("shape,density,seed", [((37, 53), 0.2, 1), ((200, 150), 0.05, 2),
                                                ((64, 64), 0.9, 3), ((1, 300), 0.5, 4)])
def test_dyadic_matches_numpy_dense_bit_exact(shape, density, seed):
    # Small-integer values and x = k / 2^10 make every partial sum exact, so
    # the oracle must equal numpy's dense product whatever order BLAS uses.
    m, n, rp, col, val = synth.tiny_random(*shape, density, seed, dyadic=True)
    x = synth.dyadic_vector(n, seed + 100)
    dense = np.zeros((m, n))
    for i in range(m):
        dense[i, col[rp[i]:rp[i + 1]]] = val[rp[i]:rp[i + 1]]
    y = oracle.spmv(rp, col, val, x)
    assert np.array_equal(y, dense @ x)
    assert np.array_equal(oracle.dense_matvec(dense, x), dense @ x)


def test_all_4x4_zero_one_patterns():
    # Every one of the 2^16 sparsity patterns of a 4x4 matrix, as one
    # block-diagonal CSR matrix, against numpy's batched dense product.
    pats = np.arange(1 << 16, dtype=np.int64)
    bits = ((pats[:, None] >> np.arange(16)) & 1).astype(bool).reshape(-1, 4, 4)
    vals = (synth.uindex(77, 0, np.arange(bits.size, dtype=np.uint64), 15) - 7).astype(np.float64)
    vals[vals == 0] = 3.0
    dense = np.where(bits, vals.reshape(bits.shape), 0.0)
    nb = dense.shape[0]
    x = synth.dyadic_vector(4 * nb, 78)
    blk_r, r, c = np.nonzero(dense)
    rows = blk_r * 4 + r
    cols = blk_r * 4 + c
    _, _, rp, col, val = synth.from_coo(rows, cols, dense[blk_r, r, c], 4 * nb, 4 * nb)
    y = oracle.spmv(rp, col, val, x)
    ref = np.einsum("bij,bj->bi", dense, x.reshape(nb, 4)).reshape(-1)
    assert np.array_equal(y, ref)


def test_matches_scipy_csr_within_bound():
    sp = pytest.importorskip("scipy.sparse")
    n, _, rp, col, val = synth.stencil27(16)
    x = synth.vector(n, 203)
    y = oracle.spmv(rp, col, val, x)
    ys = sp.csr_matrix((val, col, rp), shape=(n, n)) @ x
    ab = oracle.absax(rp, col, val, x)
    assert np.all(np.abs(y - ys) <= 1e-12 * ab)


def _exact_rows(rp, col, val, x):
    out = []
    for i in range(len(rp) - 1):
        s = Fraction(0)
        for j in range(rp[i], rp[i + 1]):
            s += Fraction(float(val[j])) * Fraction(float(x[col[j]]))
        out.append(s)
    return out


def test_dot2_and_plain_sum_against_exact_rationals():
    # Random rows of mixed magnitude with heavy cancellation: Dot2 is within
    # u|y| + n^2 u^2 |A||x| of the exact value; the storage-order sum within
    # gamma_n |A||x| (Higham, Accuracy and Stability, Sec. 3.1).
    m, n, rp, col, val = synth.tiny_random(40, 300, 0.6, 21)
    val = val * np.exp2(synth.uindex(22, 0, np.arange(val.size, dtype=np.uint64), 40) - 20)
    x = synth.vector(n, 23)
    ex = _exact_rows(rp, col, val, x)
    y2 = oracle.spmv_accurate(rp, col, val, x)
    y1 = oracle.spmv(rp, col, val, x)
    ab = oracle.absax(rp, col, val, x)
    u = 2.0 ** -53
    for i in range(m):
        k = rp[i + 1] - rp[i]
        e2 = abs(Fraction(float(y2[i])) - ex[i])
        assert e2 <= Fraction(u) * abs(ex[i]) + Fraction(k * k * u * u) * Fraction(float(ab[i])) * 2
        e1 = abs(Fraction(float(y1[i])) - ex[i])
        assert e1 <= Fraction(k * u / (1 - k * u)) * Fraction(float(ab[i]))


def test_csr_validation_cases():
    rp = np.array([0, 2, 3], dtype=np.int32)
    col = np.array([0, 1, 1], dtype=np.int32)
    assert oracle.csr_valid(2, 2, 3, rp, col)
    assert not oracle.csr_valid(2, 2, 3, np.array([1, 2, 3], dtype=np.int32), col)  # rp[0] != 0
    assert not oracle.csr_valid(2, 2, 3, np.array([0, 3, 2], dtype=np.int32), col)  # decreasing
    assert not oracle.csr_valid(2, 2, 4, rp, np.array([0, 1, 1, 0], dtype=np.int32))  # rp[N] != nnz
    assert not oracle.csr_valid(2, 2, 3, rp, np.array([0, 2, 1], dtype=np.int32))  # col >= n_cols
    assert not oracle.csr_valid(2, 2, 3, rp, np.array([0, -1, 1], dtype=np.int32))  # col < 0
    assert oracle.csr_valid(0, 0, 0, np.array([0], dtype=np.int32), np.zeros(0, dtype=np.int32))
    assert oracle.rows_sorted(rp, col)
    assert not oracle.rows_sorted(np.array([0, 2], dtype=np.int32), np.array([1, 0], dtype=np.int32))
    assert not oracle.rows_sorted(np.array([0, 2], dtype=np.int32), np.array([1, 1], dtype=np.int32))


def test_planted_mistakes_are_caught():
    # A dropped term, a transposed operand and a wrong index each break one of
    # the pins above; the pins are only worth something if that is so.
    n, _, rp, col, val = synth.laplacian2d(10)
    x = synth.dyadic_vector(n, 5)
    dense = np.zeros((n, n))
    for i in range(n):
        dense[i, col[rp[i]:rp[i + 1]]] = val[rp[i]:rp[i + 1]]
    good = oracle.spmv(rp, col, val, x)
    assert np.array_equal(good, dense @ x)
    dropped = oracle.spmv(rp, col, np.where(np.arange(val.size) == 7, 0.0, val), x)
    assert not np.array_equal(dropped, dense @ x)
    # transposed: column-wise product of a nonsymmetric matrix
    v2 = val.copy()
    v2[1] = 3.0
    dense2 = dense.copy()
    i1 = np.searchsorted(rp, 1, side="right") - 1
    dense2[i1, col[1]] = 3.0
    assert not np.array_equal(oracle.spmv(rp, col, v2, x), dense2.T @ x)
    shifted = oracle.spmv(rp, np.minimum(col + 1, n - 1).astype(np.int32), val, x)
    assert not np.array_equal(shifted, dense @ x)

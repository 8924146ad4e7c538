"""The multi-core OpenMP CSR baseline (measurement infrastructure) computes
the same products as the oracle: bit for bit on dyadic inputs (every partial
sum exact, so fused or not, any order gives the same bits), within rounding
otherwise; empty rows and trailing empty rows give +0."""
import numpy as np

import cpu_omp as omp
import oracle
import synth


def test_dyadic_bit_exact_with_empty_rows():
    for k, d in enumerate((0.0, 0.002, 0.05, 0.6)):
        n, m, rp, col, val = synth.tiny_random(900, 500, d, 40 + k, dyadic=True)
        x = synth.dyadic_vector(m, 7)
        assert np.array_equal(omp.spmv(rp, col, val, x), oracle.spmv(rp, col, val, x)), d


def test_within_rounding_on_stencil_and_rmat():
    for n, m, rp, col, val in (synth.stencil27(16), synth.rmat(12, 8, seed_edges=5, seed_vals=6)):
        x = synth.vector(m, 9)
        ref = oracle.spmv_accurate(rp, col, val, x)
        ab = oracle.absax(rp, col, val, x)
        assert np.all(np.abs(omp.spmv(rp, col, val, x) - ref) <= 1e-12 * ab + 0.0)


def test_trailing_empty_rows_and_timing():
    rp = np.array([0, 2, 2, 3, 3, 3], dtype=np.int32)
    col = np.array([0, 4, 2], dtype=np.int32)
    val = np.array([1.5, -2.0, 4.0])
    x = np.arange(5, dtype=np.float64)
    y = omp.spmv(rp, col, val, x)
    assert list(y) == [-8.0, 0.0, 8.0, 0.0, 0.0]
    assert np.all(np.signbit(y[[1, 3, 4]]) == False)
    sec, th = omp.time_spmv(rp, col, val, x, 3)
    assert sec >= 0 and th >= 1

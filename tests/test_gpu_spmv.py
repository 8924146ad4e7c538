"""GPU parity of the row-split SpMV family (Sec. II, Fig. 2; remedies of
Sec. III-E, Table II) against the CPU oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
import paper_1711_05487_amd as pkg
import synth
from spmv_cases import check_f64, check_reduced, matrix, xvec

pytestmark = pytest.mark.gpu

ROW_OPTS = [0, pkg.OPT_UNROLL, pkg.OPT_PREFETCH, pkg.OPT_DELTA,
            pkg.OPT_DELTA | pkg.OPT_PREFETCH, pkg.OPT_UNROLL | pkg.OPT_PREFETCH,
            pkg.OPT_DELTA | pkg.OPT_UNROLL]


def run(A, x, opts=None, G=0):
    if opts is not None:
        A.select("forced", forced_opts=opts, rows_per_group=G)
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    y = A.spmv(xd)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def test_laplacian_plain_matches_oracle():
    n, m, rp, col, val = matrix("lap100")
    x = xvec("lap100", m)
    A = pkg.CsrMatrix(rp, col, val)
    info = A.select("plain")
    assert info["lanes_per_row"] == 4 and info["opts"] == 0  # 2^round(log2 4.96)
    check_f64(run(A, x), rp, col, val, x, "lap100 plain")


@pytest.mark.parametrize("opts", ROW_OPTS)
@pytest.mark.parametrize("G", [1, 2, 4, 8, 16, 32, 64])
def test_dyadic_bit_exact_every_lane_count(opts, G):
    # exact arithmetic: every summation order must give the oracle's bits
    n, m, rp, col, val = synth.tiny_random(301, 257, 0.08, 7 + G, dyadic=True)
    x = synth.dyadic_vector(m, 8)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    y = run(A, x, opts, G)
    assert np.array_equal(y, oracle.spmv(rp, col, val, x))


def test_identity_permutation_bit_exact():
    n = 4099
    x = synth.vector(n, 5)
    A = pkg.CsrMatrix(np.arange(n + 1), np.arange(n), np.ones(n))
    for opts in ROW_OPTS:
        assert np.array_equal(run(A, x, opts), x)
    pi = synth.permutation(n, 6)
    P = pkg.CsrMatrix(np.arange(n + 1), pi, np.ones(n))
    for opts in (0, pkg.OPT_UNROLL, pkg.OPT_PREFETCH):
        assert np.array_equal(run(P, x, opts), x[pi])


def test_all_4x4_patterns_bit_exact():
    pats = np.arange(1 << 16, dtype=np.int64)
    bits = ((pats[:, None] >> np.arange(16)) & 1).astype(bool).reshape(-1, 4, 4)
    vals = (synth.uindex(77, 0, np.arange(bits.size, dtype=np.uint64), 15) - 7).astype(np.float64)
    vals[vals == 0] = 3.0
    dense = np.where(bits, vals.reshape(bits.shape), 0.0)
    b, r, c = np.nonzero(dense)
    nb = dense.shape[0]
    _, _, rp, col, val = synth.from_coo(b * 4 + r, b * 4 + c, dense[b, r, c], 4 * nb, 4 * nb)
    x = synth.dyadic_vector(4 * nb, 78)
    A = pkg.CsrMatrix(rp, col, val)
    want = oracle.spmv(rp, col, val, x)
    for opts in ROW_OPTS:
        for G in (1, 4, 64):
            assert np.array_equal(run(A, x, opts, G), want), (opts, G)


def test_empty_rows_zero_and_empty_matrix():
    rp = np.array([0, 0, 3, 3, 3, 5, 5], dtype=np.int32)
    col = np.array([0, 2, 4, 1, 3], dtype=np.int32)
    val = np.array([1.0, -2.0, 3.0, 4.0, -5.0])
    x = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    A = pkg.CsrMatrix(rp, col, val, n_cols=5)
    for opts in ROW_OPTS:
        y = run(A, x, opts)
        assert np.array_equal(y, oracle.spmv(rp, col, val, x))
        assert not np.signbit(y[[0, 2, 3, 5]]).any()
    E = pkg.CsrMatrix(np.zeros(1, dtype=np.int32), np.zeros(0), np.zeros(0), n_cols=3)
    xd = torch.ones(3, dtype=torch.float64, device="cuda")
    yd = torch.ones(1, dtype=torch.float64, device="cuda")[:0]
    E.spmv(xd, yd)
    Z = pkg.CsrMatrix(np.zeros(4, dtype=np.int32), np.zeros(0), np.zeros(0), n_cols=2)
    y = run(Z, np.array([1.0, 2.0]))
    assert np.array_equal(y, np.zeros(3)) and not np.signbit(y).any()


@pytest.mark.parametrize("opts", ROW_OPTS)
def test_stencil27_full_size(opts):
    n, m, rp, col, val = matrix("st27_128")
    x = xvec("st27_128", m)
    A = pkg.CsrMatrix(rp, col, val)
    info = A.select("forced", forced_opts=opts)
    if opts & pkg.OPT_DELTA:
        assert info["delta_bits"] == 16
    check_f64(run(A, x), rp, col, val, x, f"st27 opts={opts}")


def test_delta_codes_bit_exact():
    for name, w in (("lap100", 8), ("st27_24", 16)):
        n, m, rp, col, val = matrix(name)
        A = pkg.CsrMatrix(rp, col, val)
        info = A.select("forced", forced_opts=pkg.OPT_DELTA)
        assert info["delta_bits"] == w
        got = A.debug_copy(pkg.DEBUG_CODES, np.uint8 if w == 8 else np.uint16)
        assert np.array_equal(got, oracle.delta_encode(rp, col, w))
    n, m, rp, col, val = matrix("unif17")  # first offsets far beyond 16 bits
    assert oracle.delta_width(rp, col) == 32
    A = pkg.CsrMatrix(rp, col, val)
    assert A.select("forced", forced_opts=pkg.OPT_DELTA)["delta_bits"] == 32


def test_stored_values_bit_exact():
    v = np.concatenate([synth.vector(50000, 1) * np.exp2(
        synth.uindex(2, 0, np.arange(50000, dtype=np.uint64), 300) - 150),
        [1.0 + 2.0 ** -8 + 2.0 ** -40, 2.0 ** -134, 1.5 * 2.0 ** -134, (2 - 2.0 ** -8) * 2.0 ** 127,
         -0.0, np.inf, -np.inf, np.nan, 1e-310, -3.0e38]])
    n = v.size
    rp = np.arange(n + 1, dtype=np.int32)
    col = np.zeros(n, dtype=np.int32)
    for storage, dt, ref in (("f64", np.float64, v.view(np.uint64)),
                             ("f32", np.uint32, oracle.to_f32(v).view(np.uint32)),
                             ("bf16", np.uint16, oracle.to_bf16_bits(v))):
        A = pkg.CsrMatrix(rp, col, v, n_cols=1, storage=storage)
        got = A.debug_copy(pkg.DEBUG_VALUES, dt)
        if storage == "f64":
            got = got.view(np.uint64)
        assert np.array_equal(got, ref), storage


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("name", ["lap100", "st27_24"])
def test_reduced_precision_within_bound(storage, name):
    n, m, rp, col, val = matrix(name)
    x = xvec(name, m)
    A = pkg.CsrMatrix(rp, col, val, storage=storage)
    for opts in (0, pkg.OPT_DELTA, pkg.OPT_UNROLL, pkg.OPT_PREFETCH):
        A.select("forced", forced_opts=opts)
        xd = torch.from_numpy(oracle.to_f32(x)).cuda()
        y = A.spmv(xd)
        torch.cuda.synchronize()
        check_reduced(y.cpu().numpy(), rp, col, val, x, storage, f"{name} {storage} {opts}")


def test_reduced_precision_dyadic_exact():
    n, m, rp, col, val = synth.tiny_random(500, 400, 0.05, 3, dyadic=True)
    x = synth.dyadic_vector(m, 4)
    for storage in ("f32", "bf16"):
        A = pkg.CsrMatrix(rp, col, val, n_cols=m, storage=storage)
        xd = torch.from_numpy(x.astype(np.float32)).cuda()
        y = A.spmv(xd)
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy().astype(np.float64), oracle.spmv(rp, col, val, x))


def test_invalid_matrices_rejected():
    good_rp = np.array([0, 2, 3], dtype=np.int32)
    good_col = np.array([0, 1, 1], dtype=np.int32)
    v = np.ones(3)
    cases = [
        (np.array([0, 3, 2], dtype=np.int32), good_col),          # decreasing
        (np.array([1, 2, 3], dtype=np.int32), good_col),          # rp[0] != 0
        (good_rp, np.array([0, 2, 1], dtype=np.int32)),           # col >= n_cols
        (good_rp, np.array([0, -1, 1], dtype=np.int32)),          # col < 0
        (np.array([0, 9, 3], dtype=np.int32), good_col),          # rp beyond nnz
    ]
    for rp, col in cases:
        assert not oracle.csr_valid(2, 2, 3, rp, col)
        with pytest.raises(pkg.CsrError) as ei:
            pkg.CsrMatrix(rp, col, v, n_cols=2)
        assert ei.value.status == 2
    A = pkg.CsrMatrix(good_rp, good_col, v, n_cols=2)
    assert A.query()["rows_sorted"] == 1
    U = pkg.CsrMatrix(np.array([0, 2], dtype=np.int32), np.array([1, 0], dtype=np.int32),
                      np.ones(2), n_cols=2)
    assert U.query()["rows_sorted"] == 0
    assert U.select("forced", forced_opts=pkg.OPT_DELTA)["delta_bits"] == 32


def test_aliasing_rejected():
    n, m, rp, col, val = matrix("lap37")
    A = pkg.CsrMatrix(rp, col, val)
    buf = torch.zeros(2 * n, dtype=torch.float64, device="cuda")
    with pytest.raises(pkg.CsrError) as ei:
        A.spmv(buf[:n], buf[n // 2:n // 2 + n])
    assert ei.value.status == 1
    A.spmv(buf[:n], buf[n:])


def test_deterministic_run_twice():
    n, m, rp, col, val = matrix("st27_24")
    x = synth.vector(m, 3)
    A = pkg.CsrMatrix(rp, col, val)
    for opts in ROW_OPTS:
        y1 = run(A, x, opts)
        y2 = run(A, x)
        assert np.array_equal(y1.view(np.uint64), y2.view(np.uint64))


def test_triad_plausible():
    bw = pkg.triad(1 << 28, 3)
    assert 1e12 < bw < 9e12


@pytest.mark.parametrize("name", ["rmat14", "unif17", "lap100"])
def test_dynamic_rows_same_bits_as_static(name):
    """The row-split kernels' dynamic schedule (resident workgroups taking
    blocks of rows from a counter that the last one resets) sums every row
    in the same order as the static schedule: the same bits, call after
    call, and parity with the oracle."""
    n, m, rp, col, val = matrix(name)
    x = xvec(name, m)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    for opts in (0, pkg.OPT_UNROLL, pkg.OPT_PREFETCH, pkg.OPT_DECOMP, pkg.OPT_DELTA):
        A.select("forced", forced_opts=opts, long_row_floor=200)
        y_static = run(A, x)
        info = A.select("forced", forced_opts=opts, long_row_floor=200, dynamic_rows=1)
        assert info["dynamic_rows"] == 1
        y1, y2 = run(A, x), run(A, x)
        assert np.array_equal(y1.view(np.uint64), y_static.view(np.uint64)), (name, opts)
        assert np.array_equal(y2.view(np.uint64), y1.view(np.uint64)), (name, opts)
    check_f64(y1, rp, col, val, x, f"{name} dynamic rows")
    with pytest.raises(pkg.CsrError):
        A.select("forced", forced_opts=0, dynamic_rows=2)
    A.close()

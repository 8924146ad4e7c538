"""GPU parity of the nnz-balanced merge-path SpMV (IMB remedy, Sec. III-E,
Table II): the tile table bit-exact against the oracle's merge-path definition,
and y against the oracle on regular, skewed, empty-row and long-row inputs."""
import numpy as np
import pytest
import torch

import oracle
import paper_1711_05487_amd as pkg
import synth
from spmv_cases import check_f64, check_reduced, matrix, xvec

pytestmark = pytest.mark.gpu

M = pkg.OPT_MERGE
MERGE_OPTS = [M, M | pkg.OPT_PREFETCH, M | pkg.OPT_UNROLL, M | pkg.OPT_DELTA]


def run(A, x, opts=None, L=0):
    if opts is not None:
        A.select("forced", forced_opts=opts, merge_items=L)
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    y = A.spmv(xd)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def long_and_empty_rows():
    lens = [0, 0, 5000, 1, 0, 3000, 0, 0, 2, 10000, 0] + [3] * 500 + [0] * 100 + [9000]
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    col = np.concatenate([np.sort(synth.uindex(5, i, np.arange(l, dtype=np.uint64), 20000))
                          for i, l in enumerate(lens)]).astype(np.int32)
    val = (synth.uindex(6, 0, np.arange(rp[-1], dtype=np.uint64), 9) - 4).astype(float)
    return len(lens), 20000, rp, col, val


def expected_slack(rp, L):
    """Row-aligned tiles when every row has at most 63 nonzeros."""
    s = int(np.diff(rp).max(initial=0)) + 1
    return s if s <= 64 and s < L else 0


@pytest.mark.parametrize("L", [256, 512, 1024])
def test_tile_table_bit_exact(L):
    for name in ("lap100", "rmat14", "st27_24", "unif14"):
        n, m, rp, col, val = matrix(name)
        A = pkg.CsrMatrix(rp, col, val)
        info = A.select("forced", forced_opts=M, merge_items=L)
        assert info["merge_slack"] == expected_slack(rp, L), name
        ti, tj = oracle.merge_tiles(rp, L, info["merge_slack"])
        assert np.array_equal(A.debug_copy(pkg.DEBUG_TILE_I, np.int32), ti)
        assert np.array_equal(A.debug_copy(pkg.DEBUG_TILE_J, np.int32), tj)
        if info["merge_slack"]:  # no row spans two tiles
            assert np.array_equal(tj, rp[ti])


@pytest.mark.parametrize("L", [256, 512, 1024])
@pytest.mark.parametrize("opts", MERGE_OPTS)
def test_dyadic_bit_exact(opts, L):
    cases = [synth.tiny_random(700, 300, d, 11 + k, dyadic=True)
             for k, d in enumerate((0.0, 0.002, 0.02, 0.3, 0.95))]
    cases.append(long_and_empty_rows())
    for n, m, rp, col, val in cases:
        x = synth.dyadic_vector(m, 12)
        A = pkg.CsrMatrix(rp, col, val, n_cols=m)
        assert np.array_equal(run(A, x, opts, L), oracle.spmv(rp, col, val, x)), (n, opts, L)


@pytest.mark.parametrize("L", [256, 512, 1024])
def test_merge_codes_bit_exact(L):
    """MERGE|DELTA: on row-aligned tiles whose column ranges need 16 bits and
    whose windows hold at most 256 distinct columns (512 with 9-bit ranks on
    1,024-item tiles), window codes (tile bases, dictionaries, lengths or
    ninth-bit records, and ranks equal to the oracle's); otherwise tile
    bases and per-nonzero offsets at the narrowest width that holds every
    tile's column range; int32 columns when no width fits."""
    seen = set()
    for name in ("lap100", "st27_24", "rmat14", "unif14", "unif17"):
        n, m, rp, col, val = matrix(name)
        A = pkg.CsrMatrix(rp, col, val)
        info = A.select("forced", forced_opts=M | pkg.OPT_DELTA, merge_items=L)
        ti, tj = oracle.merge_tiles(rp, L, info["merge_slack"])
        want = 32
        for w in (8, 16):
            if oracle.merge_codes(tj, col, w) is not None:
                want = w
                break
        wide = L == 1024
        win = (oracle.window_codes(tj, col, 512 if wide else 256)
               if want == 16 and info["merge_slack"] > 0 else None)
        assert info["window_codes"] == (0 if win is None else 3 if wide else 1), (name, L)
        if win is not None:
            seen.add("window9" if wide else "window")
            assert info["delta_bits"] == (9 if wide else 8)
            base, wlen, dct, codes = win
            assert np.array_equal(A.debug_copy(pkg.DEBUG_TILE_BASE, np.int32), base)
            rec = oracle.window_rank_records(tj, codes, wlen, vec=2).ravel() if wide else wlen
            assert np.array_equal(A.debug_copy(pkg.DEBUG_WINDOW_LEN, np.int32), rec), (name, L)
            got = A.debug_copy(pkg.DEBUG_WINDOW_DICT, np.uint16).reshape(dct.shape)
            assert np.array_equal(got, dct), (name, L)
            assert np.array_equal(A.debug_copy(pkg.DEBUG_WINDOW_CODES, np.uint8),
                                  (codes & 255).astype(np.uint8)), (name, L)
            continue
        assert info["delta_bits"] == want, (name, L)
        if want == 32:
            seen.add("int32")
            continue
        seen.add(f"delta{want}")
        base, codes = oracle.merge_codes(tj, col, want)
        assert np.array_equal(A.debug_copy(pkg.DEBUG_TILE_BASE, np.int32), base)
        got = A.debug_copy(pkg.DEBUG_MERGE_CODES, np.uint16 if want == 16 else np.uint8)
        assert np.array_equal(got, codes), (name, L)
    if L == 1024:  # windows outgrow 256 entries: 9-bit ranks
        assert "window9" in seen
    else:
        assert "window" in seen


def test_merge_codes_same_bits_as_int32_columns():
    """The codes decode to the same columns: y is bit-identical to the int32
    merge tiles of the same size."""
    for name in ("lap100", "st27_24", "rmat14"):
        n, m, rp, col, val = matrix(name)
        x = xvec(name, m)
        A = pkg.CsrMatrix(rp, col, val)
        for L in (256, 512, 1024):
            info = A.select("forced", forced_opts=M | pkg.OPT_DELTA, merge_items=L)
            assert info["delta_bits"] in (8, 9, 16)
            y_codes = run(A, x)
            y_i32 = run(A, x, M | pkg.OPT_PREFETCH, L)
            assert np.array_equal(y_codes.view(np.uint64), y_i32.view(np.uint64)), (name, L)


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
    for L in (256, 512, 1024):
        assert np.array_equal(run(A, x, M, L), want)


@pytest.mark.parametrize("name", ["rmat14", "st27_24", "lap100"])
def test_random_values_within_bound(name):
    n, m, rp, col, val = matrix(name)
    x = xvec(name, m)
    A = pkg.CsrMatrix(rp, col, val)
    for opts in MERGE_OPTS:
        check_f64(run(A, x, opts), rp, col, val, x, f"{name} {opts}")


def test_long_rows_random_values():
    n, m, rp, col, _ = long_and_empty_rows()
    val = synth.um11(8, 0, np.arange(len(col), dtype=np.uint64))
    x = synth.vector(m, 9)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    for L in (256, 512, 1024):
        check_f64(run(A, x, M, L), rp, col, val, x, f"long rows L={L}")


def test_stencil27_full_size():
    n, m, rp, col, val = matrix("st27_128")
    x = xvec("st27_128", m)
    A = pkg.CsrMatrix(rp, col, val)
    for opts in MERGE_OPTS:
        check_f64(run(A, x, opts), rp, col, val, x, f"st27 {opts}")


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_reduced_precision(storage):
    for name in ("rmat14", "st27_24"):
        n, m, rp, col, val = matrix(name)
        x = xvec(name, m)
        A = pkg.CsrMatrix(rp, col, val, storage=storage)
        for L in (256, 1024):
            A.select("forced", forced_opts=M, merge_items=L)
            y = A.spmv(torch.from_numpy(oracle.to_f32(x)).cuda())
            torch.cuda.synchronize()
            check_reduced(y.cpu().numpy(), rp, col, val, x, storage, f"{name} {storage} L={L}")


def test_invalid_tile_size_rejected():
    """Tile sizes are multiples of 256 from 256 to 2048 (other than 256,
    512 and 1024 compiled at run time)."""
    n, m, rp, col, val = matrix("lap37")
    A = pkg.CsrMatrix(rp, col, val)
    for L in (128, 640, 2304, 4096):
        with pytest.raises(pkg.CsrError):
            A.select("forced", forced_opts=M, merge_items=L)


def test_deterministic():
    n, m, rp, col, val = matrix("rmat14")
    x = synth.vector(m, 4)
    A = pkg.CsrMatrix(rp, col, val)
    for L in (256, 512):
        y1 = run(A, x, M, L)
        y2 = run(A, x)
        assert np.array_equal(y1.view(np.uint64), y2.view(np.uint64))


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_window_codes_parity(storage):
    """Window-coded tiles against the oracle, with empty rows and tiles
    (rows of a banded matrix removed in runs), in every value storage."""
    n, m, rp, col, val = matrix("st27_24")
    keep = np.ones(n, dtype=bool)
    for k in range(0, n, 997):
        keep[k:k + 40] = False  # runs of emptied rows, some longer than a tile's rows
    lens = np.where(keep, np.diff(rp), 0)
    rows = np.repeat(np.arange(n), np.diff(rp))
    sel = keep[rows]
    rp2 = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    col2, val2 = col[sel], val[sel]
    x = xvec("st27_24", m)
    A = pkg.CsrMatrix(rp2, col2, val2, n_cols=m, storage=storage)
    info = A.select("forced", forced_opts=M | pkg.OPT_DELTA, merge_items=512)
    assert info["window_codes"] == 1
    if storage == "f64":
        y = run(A, x)
        check_f64(y, rp2, col2, val2, x, "window codes with empty rows")
        # the window ranks decode to the same columns: bit-identical to int32 tiles
        y_i32 = run(A, x, M | pkg.OPT_PREFETCH, 512)
        assert np.array_equal(y.view(np.uint64), y_i32.view(np.uint64))
        assert np.all(y[~keep] == 0)
    else:
        xs = torch.from_numpy(oracle.to_f32(x)).cuda()
        y = A.spmv(xs)
        torch.cuda.synchronize()
        check_reduced(y.cpu().numpy(), rp2, col2, val2, x, storage, f"window codes {storage}")


def _dyadic(val, seed):
    """Small integers (exact products and sums with a dyadic x)."""
    q = synth.uindex(seed, 0, np.arange(len(val), dtype=np.uint64), 15).astype(np.float64) - 7.0
    q[q == 0] = 3.0
    return q


@pytest.mark.parametrize("L", [256, 512])
def test_column_blocks_bit_exact(L):
    """MERGE on short rows spread over an x above one XCD's L2: column blocks
    equal to the oracle's (row pointers, columns, values), and y from one
    pass per block equals the oracle bit for bit on dyadic inputs."""
    n, m, rp, col, val = matrix("unif600k")
    val = _dyadic(val, 41)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    info = A.select("forced", forced_opts=M, merge_items=L)
    B = info["column_blocks"]
    assert B == 3  # 4.8 MB of x in slabs of at most 2 MiB
    width = (m + B - 1) // B
    rpb, colb, valb = oracle.column_blocks(rp, col, val, B, width)
    assert np.array_equal(A.debug_copy(pkg.DEBUG_CB_ROWPTR, np.int32), rpb.ravel())
    assert np.array_equal(A.debug_copy(pkg.DEBUG_CB_COL, np.int32), colb)
    assert np.array_equal(A.debug_copy(pkg.DEBUG_CB_VAL, np.float64), valb)
    x = synth.dyadic_vector(m, 42)
    assert np.array_equal(run(A, x), oracle.spmv(rp, col, val, x))
    # blocks are deterministic: a second product gives the same bits
    assert np.array_equal(run(A, x), run(A, x))
    A.close()


@pytest.fixture(scope="module")
def rmat21():
    return synth.rmat(21, 16)


def test_column_blocks_with_split_rows(rmat21):
    """Skewed rows (R-MAT scale 21: rows of thousands of nonzeros, so the
    tiles are not row-aligned and rows span tiles) over an x above one XCD's
    L2: one pass per column block, each with its carries; blocks equal to the
    oracle's, y bit-exact on dyadic inputs and deterministic, and within the
    FP64 bar on the generator's values."""
    n, m, rp, col, val = rmat21
    dv = _dyadic(val, 43)
    A = pkg.CsrMatrix(rp, col, dv, n_cols=m)
    # on tiles that are not row-aligned unless turned off
    assert A.select("forced", forced_opts=M, merge_items=512, split_row_blocks=0)["column_blocks"] == 0
    for opts in (M, M | pkg.OPT_DELTA):  # no eligible codes: the same blocks
        info = A.select("forced", forced_opts=opts, merge_items=512, split_row_blocks=1)
        assert info["merge_slack"] == 0 and info["delta_bits"] == 32
        assert info["column_blocks"] == 8  # 16 MB of x in slabs of at most 2 MiB
    B = 8
    width = (m + B - 1) // B
    rpb, colb, valb = oracle.column_blocks(rp, col, dv, B, width)
    assert np.array_equal(A.debug_copy(pkg.DEBUG_CB_ROWPTR, np.int32), rpb.ravel())
    assert np.array_equal(A.debug_copy(pkg.DEBUG_CB_COL, np.int32), colb)
    assert np.array_equal(A.debug_copy(pkg.DEBUG_CB_VAL, np.float64), valb)
    rows, ptr = oracle.column_block_rows(rpb)  # blocks after the first: row lists
    assert rows.size < (B - 1) * n
    assert np.array_equal(A.debug_copy(pkg.DEBUG_CB_ROWS, np.int32), rows)
    assert np.array_equal(A.debug_copy(pkg.DEBUG_CB_ROWLIST_PTR, np.int32), ptr)
    x = synth.dyadic_vector(m, 44)
    y = run(A, x)
    assert np.array_equal(y, oracle.spmv(rp, col, dv, x))
    assert np.array_equal(run(A, x), y)
    A.close()
    xr = synth.vector(m, 45)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    assert A.select("forced", forced_opts=M, merge_items=1024,
                    split_row_blocks=1)["column_blocks"] == 8
    check_f64(run(A, xr), rp, col, val, xr, "rmat21 column blocks")
    A.close()


def _wide(n_rows=200_000, n_cols=1_500_000, k=8, seed=51):
    """Rectangular, 8 random columns per row (repeats allowed, summed in
    storage order): x of 12 MB (f64) or 6 MB (f32)."""
    idx = np.arange(n_rows * k, dtype=np.uint64)
    cols = synth.uindex(seed, 0, idx, n_cols).reshape(n_rows, k).astype(np.int64)
    cols.sort(axis=1)
    rp = np.arange(0, n_rows * k + 1, k, dtype=np.int32)
    return n_rows, n_cols, rp, cols.ravel().astype(np.int32), synth.u01(seed, 1, idx)


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_column_blocks_parity(storage):
    n, m, rp, col, val = _wide()
    x = synth.vector(m, 52)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m, storage=storage)
    info = A.select("forced", forced_opts=M | pkg.OPT_PREFETCH)
    assert info["column_blocks"] == (6 if storage == "f64" else 3)
    if storage == "f64":
        check_f64(run(A, x), rp, col, val, x, "column blocks")
    else:
        xs = torch.from_numpy(oracle.to_f32(x)).cuda()
        y = A.spmv(xs)
        torch.cuda.synchronize()
        check_reduced(y.cpu().numpy(), rp, col, val, x, storage, f"column blocks {storage}")
    # codes take the single pass; without eligible codes (these rows' column
    # ranges need 32 bits) MERGE|DELTA keeps the column blocks
    info = A.select("forced", forced_opts=M | pkg.OPT_DELTA)
    assert info["delta_bits"] == 32
    assert info["column_blocks"] == (6 if storage == "f64" else 3)
    if storage == "f64":
        check_f64(run(A, x), rp, col, val, x, "column blocks, codes not eligible")
    A.close()
    # x inside one L2, or rows whose columns stay close: a single pass
    for name in ("unif17", "st27_128"):
        n, m, rp, col, val = matrix(name)
        B = pkg.CsrMatrix(rp, col, val, n_cols=m)
        assert B.select("forced", forced_opts=M | pkg.OPT_PREFETCH)["column_blocks"] == 0, name
        assert B.select("forced", forced_opts=M)["column_blocks"] == 0, name
        B.close()


def far_bidiagonal(n, seed, offset=1000):
    """a_ii and a_i,i+offset: about 127 rows per 256-item tile (more rows than
    lanes), a column range above 2^8 (16-bit codes) and at most 256 distinct
    columns per tile (window codes)."""
    i = np.arange(n)
    rows = np.concatenate([i, i[:-offset]])
    cols = np.concatenate([i, i[:-offset] + offset])
    vals = _dyadic(np.zeros(rows.size), seed)
    return synth.from_coo(rows, cols, vals, n, n)


def test_window_codes_many_rows_per_tile():
    """Window-coded tiles holding more rows than lanes: with dyadic values
    and x, the same bits as int32 columns on the same tiles and as the
    oracle."""
    n, m, rp, col, val = far_bidiagonal(300_001, 12)
    x = synth.dyadic_vector(m, 14)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    info = A.select("forced", forced_opts=M | pkg.OPT_DELTA, merge_items=256)
    assert info["window_codes"] == 1
    y_w = run(A, x)
    y_i = run(A, x, M | pkg.OPT_PREFETCH, 256)
    assert np.array_equal(y_w.view(np.uint64), y_i.view(np.uint64))
    assert np.array_equal(y_w, oracle.spmv(rp, col, val, x))


@pytest.mark.parametrize("name", ["st27_24", "bidiag"])
def test_window_runs_bit_exact_and_same_bits(name):
    """Run windows (window codes whose windows are at most 14 runs of
    consecutive columns): records bit-exact against the oracle's, and y
    bit-identical to the dictionary form and to int32 columns on the same
    tiles (dyadic values: equal to the oracle)."""
    if name == "bidiag":
        n, m, rp, col, val = far_bidiagonal(200_003, 17)
        L = 256
    else:
        n, m, rp, col, val = matrix(name)
        val = _dyadic(val, 18)
        L = 512
    x = synth.dyadic_vector(m, 19)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    info = A.select("forced", forced_opts=M | pkg.OPT_DELTA, merge_items=L, window_runs=1)
    s = expected_slack(rp, L)
    ti, tj = oracle.merge_tiles(rp, L, s)
    want = oracle.window_runs(tj, col)
    assert want is not None and info["window_codes"] == 2
    rec = A.debug_copy(pkg.DEBUG_WINDOW_RUNS, np.int32).reshape(-1, 16)
    assert np.array_equal(rec, want[0])
    assert np.array_equal(A.debug_copy(pkg.DEBUG_WINDOW_CODES, np.uint8), want[1])
    y_r = run(A, x)
    info = A.select("forced", forced_opts=M | pkg.OPT_DELTA, merge_items=L)
    assert info["window_codes"] == 1
    y_w = run(A, x)
    y_i = run(A, x, M | pkg.OPT_PREFETCH, L)
    assert np.array_equal(y_r.view(np.uint64), y_w.view(np.uint64))
    assert np.array_equal(y_r.view(np.uint64), y_i.view(np.uint64))
    assert np.array_equal(y_r, oracle.spmv(rp, col, val, x))


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_window_runs_parity_with_empty_rows(storage):
    """Run windows with runs of emptied rows (five every 997 rows, which
    keeps every tile within 14 runs), against the oracle in every value
    storage."""
    n, m, rp, col, val = matrix("st27_24")
    keep = np.ones(n, dtype=bool)
    for k in range(0, n, 997):
        keep[k:k + 5] = False
    lens = np.where(keep, np.diff(rp), 0)
    sel = keep[np.repeat(np.arange(n), np.diff(rp))]
    rp2 = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    col2, val2 = col[sel], val[sel]
    x = xvec("st27_24", m)
    A = pkg.CsrMatrix(rp2, col2, val2, n_cols=m, storage=storage)
    info = A.select("forced", forced_opts=M | pkg.OPT_DELTA, merge_items=512, window_runs=1)
    assert info["window_codes"] == 2
    if storage == "f64":
        y = run(A, x)
        check_f64(y, rp2, col2, val2, x, "run windows with empty rows")
        assert np.all(y[~keep] == 0)
    else:
        y = A.spmv(torch.from_numpy(oracle.to_f32(x)).cuda())
        torch.cuda.synchronize()
        check_reduced(y.cpu().numpy(), rp2, col2, val2, x, storage, f"run windows {storage}")


def tridiagonal(n, seed):
    """a_i,i-1, a_ii, a_i,i+1 with dyadic values: about 256 rows and 258
    distinct columns per 1,024-item tile (more rows than lanes, ranks past
    255)."""
    i = np.arange(n)
    rows = np.concatenate([i[1:], i, i[:-1]])
    cols = np.concatenate([i[1:] - 1, i, i[:-1] + 1])
    vals = _dyadic(np.zeros(rows.size), seed)
    return synth.from_coo(rows, cols, vals, n, n)


def _stencil_dyadic():
    n, m, rp, col, val = synth.stencil27(24)
    return n, m, rp, col, _dyadic(val, 61)


@pytest.mark.parametrize("name", ["st27_24", "tridiag"])
def test_window_codes_nine_bit_bit_exact(name):
    """9-bit window ranks on 1,024-item tiles (windows of up to 512 columns):
    tile table, bases, dictionaries, codes and ninth-bit records bit-exact
    against the oracle; y bit-exact on dyadic inputs and the same bits as
    int32 columns on the same tiles; the tridiagonal's tiles end about 256
    rows (row ends past the first 64 are read in the row-sum phase)."""
    n, m, rp, col, val = _stencil_dyadic() if name == "st27_24" else tridiagonal(300_001, 62)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    info = A.select("forced", forced_opts=M | pkg.OPT_DELTA, merge_items=1024)
    assert info["window_codes"] == 3 and info["delta_bits"] == 9
    ti, tj = oracle.merge_tiles(rp, 1024, info["merge_slack"])
    assert np.array_equal(A.debug_copy(pkg.DEBUG_TILE_I, np.int32), ti)
    assert np.array_equal(A.debug_copy(pkg.DEBUG_TILE_J, np.int32), tj)
    base, wlen, dct, ranks = oracle.window_codes(tj, col, 512)
    assert ranks.max() >= 256
    if name == "tridiag":
        assert (np.diff(ti) > 64).mean() > 0.9
    assert np.array_equal(A.debug_copy(pkg.DEBUG_TILE_BASE, np.int32), base)
    assert np.array_equal(A.debug_copy(pkg.DEBUG_WINDOW_DICT, np.uint16), dct.ravel())
    assert np.array_equal(A.debug_copy(pkg.DEBUG_WINDOW_CODES, np.uint8), (ranks & 255).astype(np.uint8))
    rec = oracle.window_rank_records(tj, ranks, wlen, vec=2)
    assert np.array_equal(A.debug_copy(pkg.DEBUG_WINDOW_LEN, np.int32), rec.ravel())
    x = synth.dyadic_vector(m, 63)
    y = run(A, x)
    assert np.array_equal(y, oracle.spmv(rp, col, val, x))
    assert np.array_equal(run(A, x, M, 1024), y)  # int32 columns, same tiles
    A.close()


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_window_codes_nine_bit_reduced_precision(storage):
    n, m, rp, col, val = synth.stencil27(24)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m, storage=storage)
    info = A.select("forced", forced_opts=M | pkg.OPT_DELTA, merge_items=1024)
    assert info["window_codes"] == 3
    ti, tj = oracle.merge_tiles(rp, 1024, info["merge_slack"])
    base, wlen, dct, ranks = oracle.window_codes(tj, col, 512)
    rec = oracle.window_rank_records(tj, ranks, wlen, vec=4)
    assert np.array_equal(A.debug_copy(pkg.DEBUG_WINDOW_LEN, np.int32), rec.ravel())
    x = synth.vector(m, 64)
    xs = torch.from_numpy(oracle.to_f32(x)).cuda()
    y = A.spmv(xs)
    torch.cuda.synchronize()
    check_reduced(y.cpu().numpy(), rp, col, val, x, storage, f"9-bit windows {storage}")
    A.close()

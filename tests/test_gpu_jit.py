"""GPU parity of the merge-path kernel compiled at run time (the paper's
just-in-time code generation, Sec. IV-D) for tile sizes outside the
prebuilt 256, 512 and 1024: tile tables and codes bit-exact against the
oracle, y bit-exact on dyadic inputs and within the FP64 / reduced-precision
bounds otherwise, on row-aligned tiles, tiles with carries (long rows),
merge and window codes, and column blocks."""
import numpy as np
import pytest
import torch

import oracle
import paper_1711_05487_amd as pkg
import synth
from spmv_cases import check_f64, check_reduced, matrix, xvec
from test_gpu_merge import MERGE_OPTS, _dyadic, expected_slack, long_and_empty_rows, run

pytestmark = pytest.mark.gpu

M = pkg.OPT_MERGE
JIT_SIZES = [768, 1536, 2048]


def codes_fit(L, code_bytes):
    b = L // 64 * code_bytes
    return b in (2, 4, 8) if b < 16 else b % 16 == 0


@pytest.mark.parametrize("L", JIT_SIZES)
def test_tile_table_bit_exact(L):
    for name in ("lap100", "rmat14", "st27_24", "unif14"):
        n, m, rp, col, val = matrix(name)
        A = pkg.CsrMatrix(rp, col, val)
        info = A.select("forced", forced_opts=M, merge_items=L)
        assert info["jit"] == 1 and info["merge_items"] == L
        assert info["merge_slack"] == expected_slack(rp, L), name
        ti, tj = oracle.merge_tiles(rp, L, info["merge_slack"])
        assert np.array_equal(A.debug_copy(pkg.DEBUG_TILE_I, np.int32), ti)
        assert np.array_equal(A.debug_copy(pkg.DEBUG_TILE_J, np.int32), tj)
        A.close()


@pytest.mark.parametrize("L", JIT_SIZES)
@pytest.mark.parametrize("opts", MERGE_OPTS)
def test_dyadic_bit_exact(opts, L):
    cases = [synth.tiny_random(700, 300, d, 11 + k, dyadic=True)
             for k, d in enumerate((0.0, 0.002, 0.02, 0.3, 0.95))]
    cases.append(long_and_empty_rows())
    for n, m, rp, col, val in cases:
        x = synth.dyadic_vector(m, 12)
        A = pkg.CsrMatrix(rp, col, val, n_cols=m)
        assert np.array_equal(run(A, x, opts, L), oracle.spmv(rp, col, val, x)), (n, opts, L)
        assert A.info["jit"] == 1
        A.close()


@pytest.mark.parametrize("L", JIT_SIZES)
def test_codes_bit_exact(L):
    """MERGE|DELTA at a run-time tile size: window codes, merge codes or int32
    columns as at the prebuilt sizes, restricted to code widths whose IPT
    codes per lane form whole loads (768: none; 1536: 16-bit; 2048: all)."""
    for name in ("lap100", "st27_24", "rmat14", "unif14"):
        n, m, rp, col, val = matrix(name)
        x = xvec(name, m)
        A = pkg.CsrMatrix(rp, col, val)
        info = A.select("forced", forced_opts=M | pkg.OPT_DELTA, merge_items=L)
        ti, tj = oracle.merge_tiles(rp, L, info["merge_slack"])
        narrow = next((w for w in (8, 16) if oracle.merge_codes(tj, col, w) is not None), 32)
        win = (oracle.window_codes(tj, col)
               if narrow == 16 and info["merge_slack"] > 0 and codes_fit(L, 1) else None)
        if win is not None:
            assert info["window_codes"] == 1 and info["delta_bits"] == 8, (name, L)
            base, wlen, dct, codes = win
            assert np.array_equal(A.debug_copy(pkg.DEBUG_TILE_BASE, np.int32), base)
            assert np.array_equal(A.debug_copy(pkg.DEBUG_WINDOW_LEN, np.int32), wlen)
            assert np.array_equal(A.debug_copy(pkg.DEBUG_WINDOW_CODES, np.uint8), codes)
        elif narrow < 32 and codes_fit(L, narrow // 8):
            assert info["window_codes"] == 0 and info["delta_bits"] == narrow, (name, L)
            base, codes = oracle.merge_codes(tj, col, narrow)
            got = A.debug_copy(pkg.DEBUG_MERGE_CODES, np.uint16 if narrow == 16 else np.uint8)
            assert np.array_equal(got, codes), (name, L)
        else:
            assert info["delta_bits"] == 32, (name, L)
        # the codes decode to the same columns: bit-identical to int32 tiles
        y_codes = run(A, x)
        y_i32 = run(A, x, M | pkg.OPT_PREFETCH, L)
        assert np.array_equal(y_codes.view(np.uint64), y_i32.view(np.uint64)), (name, L)
        check_f64(y_codes, rp, col, val, x, f"{name} L={L} codes")
        A.close()


@pytest.mark.parametrize("L", [768, 1536])
@pytest.mark.parametrize("name", ["rmat14", "st27_24", "lap100"])
def test_random_values_within_bound(name, L):
    n, m, rp, col, val = matrix(name)
    x = xvec(name, m)
    A = pkg.CsrMatrix(rp, col, val)
    for opts in (M, M | pkg.OPT_PREFETCH):
        check_f64(run(A, x, opts, L), rp, col, val, x, f"{name} L={L} opts={opts}")
    A.close()


def test_long_rows_with_carries():
    n, m, rp, col, val = long_and_empty_rows()
    val = synth.vector(len(val), 7)
    x = synth.vector(m, 8)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    for L in JIT_SIZES:
        info = A.select("forced", forced_opts=M, merge_items=L)
        assert info["merge_slack"] == 0 and info["jit"] == 1
        check_f64(run(A, x), rp, col, val, x, f"long rows L={L}")
    A.close()


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_reduced_precision(storage):
    for name in ("st27_24", "rmat14"):
        n, m, rp, col, val = matrix(name)
        x = xvec(name, m)
        A = pkg.CsrMatrix(rp, col, val, storage=storage)
        xs = torch.from_numpy(oracle.to_f32(x)).cuda()
        for L in (768, 2048):
            for opts in (M, M | pkg.OPT_DELTA):
                A.select("forced", forced_opts=opts, merge_items=L)
                y = A.spmv(xs)
                torch.cuda.synchronize()
                check_reduced(y.cpu().numpy(), rp, col, val, x, storage, f"{name} {storage} L={L}")
        A.close()


def test_column_blocks_bit_exact():
    """Column blocks at a run-time tile size (one pass per slab, each adding
    into y): bit-exact against the oracle on dyadic inputs."""
    n, m, rp, col, val = matrix("unif600k")
    val = _dyadic(val, 41)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    info = A.select("forced", forced_opts=M, merge_items=768)
    assert info["column_blocks"] == 3 and info["jit"] == 1
    x = synth.dyadic_vector(m, 42)
    assert np.array_equal(run(A, x), oracle.spmv(rp, col, val, x))
    A.close()


def test_deterministic_and_prebuilt_flag():
    n, m, rp, col, val = matrix("rmat14")
    x = synth.vector(m, 4)
    A = pkg.CsrMatrix(rp, col, val)
    y1 = run(A, x, M, 1536)
    y2 = run(A, x)
    assert np.array_equal(y1.view(np.uint64), y2.view(np.uint64))
    assert A.select("forced", forced_opts=M, merge_items=512)["jit"] == 0
    A.close()


def test_autotuner_tries_run_time_sizes():
    """jit_tiles = 1: the profile-guided autotuner also times 768 and 1536;
    whatever it keeps is correct."""
    n, m, rp, col, val = matrix("rmat14")
    x = xvec("rmat14", m)
    A = pkg.CsrMatrix(rp, col, val)
    info = A.select("profile", jit_tiles=1)
    if info["opts"] & M:
        assert info["merge_items"] in (256, 512, 768, 1024, 1536)
        assert info["jit"] == int(info["merge_items"] in (768, 1536))
    check_f64(run(A, x), rp, col, val, x, "profile with run-time tile sizes")
    A.close()

"""Full-size parity at the benchmark configurations, in the launch
configurations the benchmark times:

  C1  2-D 5-point Laplacian 100^2 (cache-resident, launch bound)
  C2  27-point stencil on 128^3 (HBM bound, the headline workload)
  C3a R-MAT scale 22, edge factor 16 (skewed rows: merge path, long rows),
      and its seeded symmetric permutation (column blocks over row lists)
  C3b uniform random 2^20 x 16 (gather bound)
  C4  FP32 / BF16 value storage of C1 and C2

Each case runs the learned and the profile-guided selection (Sec. III-E,
IV) and every merge-path tile size, and compares every row with the oracle
(FP64: |y - y_acc| <= 1e-12 (|A||x|)_i against the compensated product;
FP32/BF16: the gamma bound of the stored values)."""
import json
import os

import pytest
import torch

import oracle
import paper_1711_05487_amd as pkg
from paper_1711_05487_amd import learn
from spmv_cases import check_f64, check_reduced, matrix, xvec

pytestmark = pytest.mark.gpu

CONFIGS = ["lap100", "st27_128", "rmat22", "rmat22perm", "unif20"]


@pytest.fixture(scope="module", autouse=True)
def learned_model():
    assert os.path.exists(learn.WEIGHTS), "the committed selector model is missing"
    learn.install()
    yield


def spmv(A, x):
    y = A.spmv(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("mode", ["learned", "profile"])
@pytest.mark.parametrize("name", CONFIGS)
def test_selected_plan_full_size(name, mode):
    n, m, rp, col, val = matrix(name)
    x = xvec(name, m)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    info = A.select(mode)
    assert not info["fallback"]
    check_f64(spmv(A, x), rp, col, val, x, f"{name} {mode} opts={info['opts']}")
    A.close()


@pytest.mark.parametrize("name", ["st27_128", "rmat22", "unif20"])
def test_merge_tile_sizes_full_size(name):
    n, m, rp, col, val = matrix(name)
    x = xvec(name, m)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    for L in (256, 512, 1024):
        A.select("forced", forced_opts=pkg.OPT_MERGE | pkg.OPT_PREFETCH, merge_items=L)
        check_f64(spmv(A, x), rp, col, val, x, f"{name} merge L={L}")
    A.close()


def test_column_blocks_uniform_full_size():
    """C3b with PREFETCH|MERGE: 8 MB of x in four slabs, one pass each."""
    n, m, rp, col, val = matrix("unif20")
    x = xvec("unif20", m)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    info = A.select("forced", forced_opts=pkg.OPT_MERGE | pkg.OPT_PREFETCH)
    assert info["column_blocks"] == 4
    check_f64(spmv(A, x), rp, col, val, x, "unif20 column blocks")
    A.close()


@pytest.mark.parametrize("name", ["rmat22", "rmat22perm"])
def test_rmat_merge_plans_full_size(name):
    """R-MAT 22 and its permutation under the merge plans the irregular
    benchmark times: one pass (plain and streaming loads, split rows
    carried through the fixup) and column blocks over row lists."""
    n, m, rp, col, val = matrix(name)
    x = xvec(name, m)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    for opts, over in ((pkg.OPT_MERGE, {"split_row_blocks": 0}),
                       (pkg.OPT_MERGE | pkg.OPT_PREFETCH, {"split_row_blocks": 0}),
                       (pkg.OPT_MERGE, {})):
        info = A.select("forced", forced_opts=opts, **over)
        assert info["column_blocks"] == (0 if over else 8), info
        check_f64(spmv(A, x), rp, col, val, x, f"{name} opts={opts} {over}")
    A.close()


def test_long_row_decomposition_rmat22():
    n, m, rp, col, val = matrix("rmat22")
    x = xvec("rmat22", m)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    info = A.select("forced", forced_opts=pkg.OPT_DECOMP)
    assert info["n_long_rows"] > 0
    check_f64(spmv(A, x), rp, col, val, x, "rmat22 decomposition")
    A.close()


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("name", ["lap100", "st27_128"])
def test_reduced_precision_full_size(name, storage):
    n, m, rp, col, val = matrix(name)
    x = xvec(name, m)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m, storage=storage)
    for mode in ("learned", "plain"):
        A.select(mode)
        y = spmv(A, oracle.to_f32(x))
        check_reduced(y, rp, col, val, x, storage, f"{name} {storage} {mode}")
    A.close()


SWEEP = {}


@pytest.mark.parametrize("index", ["int32", "delta"])
@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("name", ["lap100", "st27_128"])
def test_precision_sweep_against_oracle(name, storage, index):
    """The precision sweep of the benchmark's C4 cases (merge-path tiles with
    int32 columns, then with the MB remedy's codes), each result checked at
    its bar and its error against the FP64 oracle reported: max and 99th
    percentile over rows of |y - y_acc| / (|A||x|)_i. With CSRSPMV_REPORT_DIR
    set, the table is written to precision_sweep.json there."""
    n, m, rp, col, val = matrix(name)
    x = xvec(name, m)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m, storage=storage)
    opts = pkg.OPT_MERGE | (pkg.OPT_PREFETCH if index == "int32" else pkg.OPT_DELTA)
    info = A.select("forced", forced_opts=opts)
    if index == "delta":
        assert info["delta_bits"] in (8, 9, 16)
    xin = x if storage == "f64" else oracle.to_f32(x)
    y = spmv(A, xin)
    A.close()
    what = f"{name} {storage} {index}"
    if storage == "f64":
        check_f64(y, rp, col, val, x, what)
        rep = oracle.rel_error_report(y, oracle.spmv_accurate(rp, col, val, x),
                                      oracle.absax(rp, col, val, x))
    else:
        rep = check_reduced(y, rp, col, val, x, storage, what)
    assert rep["zero_rows_exact"]
    SWEEP[what] = {"index": ("window8 runs" if info["window_codes"] == 2 else
                             f"window{info['delta_bits']}" if info["window_codes"] else
                             "int32" if info["delta_bits"] == 32 else f"delta{info['delta_bits']}"),
                   "max_rel_err": rep["max"], "p99_rel_err": rep["p99"]}
    out = os.environ.get("CSRSPMV_REPORT_DIR")
    if out:
        os.makedirs(out, exist_ok=True)
        with open(os.path.join(out, "precision_sweep.json"), "w") as f:
            json.dump(SWEEP, f, indent=1, sort_keys=True)

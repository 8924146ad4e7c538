"""GPU parity of the selection machinery: features (Sec. III-D, Table I), the
micro-benchmark probes and the profile-guided rule (Sec. III-B/C, Fig. 4),
the class-to-optimization map (Table II), the long-row decomposition
(Sec. III-E, Figs. 5-6) and the exhaustive catalogue sweep (Sec. IV-D)."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1711_05487_amd as pkg
import synth
from spmv_cases import check_f64, matrix, xvec

pytestmark = pytest.mark.gpu

F = {name: k for k, name in enumerate(oracle.FEATURE_NAMES)}


def unsorted_with_empty_rows():
    m, n = 300, 500
    lens = synth.uindex(31, 0, np.arange(m, dtype=np.uint64), 40)
    lens[::7] = 0
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    col = synth.uindex(32, 0, np.arange(rp[-1], dtype=np.uint64), n).astype(np.int32)
    val = synth.vector(rp[-1], 33)
    return m, n, rp, col, val


FEATURE_CASES = ["lap100", "st27_24", "rmat14", "unif14", "tiny", "unsorted", "onerow"]


def feature_case(name):
    if name == "tiny":
        return synth.tiny_random(333, 777, 0.03, 5)
    if name == "unsorted":
        return unsorted_with_empty_rows()
    if name == "onerow":
        return 1, 50, np.array([0, 4], dtype=np.int32), np.array([3, 4, 5, 40], dtype=np.int32), np.ones(4)
    return matrix(name)


@pytest.mark.parametrize("name", FEATURE_CASES)
def test_features_match_oracle(name):
    n, m, rp, col, val = feature_case(name)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    f, isum, sorted_flag = A.inspect()
    rf, ri = oracle.features(n, m, rp, col)
    assert np.array_equal(isum, ri)                       # exact integer sums
    assert sorted_flag == int(oracle.rows_sorted(rp, col))
    for k in ("N", "nnz_min", "nnz_max", "bw_min", "bw_max", "size", "x_reuse"):
        assert f[F[k]] == rf[F[k]], k                     # exact
    N = max(n, 1)
    gam = 2 * N * 2.0 ** -53 / (1 - 2 * N * 2.0 ** -53)   # two summation orders of N terms
    for k in ("nnz_avg", "bw_avg", "misses_avg", "mean_col_gap", "clustering_avg", "scatter_avg"):
        assert math.isclose(f[F[k]], rf[F[k]], rel_tol=max(gam, 1e-13), abs_tol=1e-300), k
    # standard deviations: the oracle's two-pass definition against exact
    # integer variances (nnz, bw) and a Welford/Chan merge (scatter)
    for k, scale in (("nnz_sd", "nnz_avg"), ("bw_sd", "bw_avg"), ("scatter_sd", "scatter_avg")):
        assert math.isclose(f[F[k]], rf[F[k]], rel_tol=1e-10, abs_tol=1e-12 * max(rf[F[scale]], 1.0)), k


def test_features_stencil27_full_size():
    n, m, rp, col, val = matrix("st27_128")
    A = pkg.CsrMatrix(rp, col, val)
    f, isum, _ = A.inspect()
    rf, ri = oracle.features(n, m, rp, col)
    assert np.array_equal(isum, ri)
    # integer-valued features exactly; the others within 2 gamma_N of the
    # oracle's: its sequential FP64 sums over N = 2,097,152 rows are only
    # accurate to gamma_N = N u / (1 - N u) ~ 2.3e-10 relative (sums of
    # non-negative terms; the deviations' two passes likewise), so two
    # summation orders may differ by 2 gamma_N. A fixed 1e-12 bar is below
    # the oracle's own error at this size (measured: up to 5.3e-11).
    for k in ("N", "nnz_min", "nnz_max", "bw_min", "bw_max", "size", "x_reuse",
              "nnz_avg", "bw_avg", "misses_avg", "mean_col_gap"):
        assert f[F[k]] == rf[F[k]], k
    u = 2.0 ** -53
    gam = 2 * n * u / (1 - n * u)
    rel = np.abs(f - rf) / np.maximum(np.abs(rf), 1e-300)
    print("full-size feature rel errors:", {oracle.FEATURE_NAMES[k]: float(rel[k]) for k in range(16)})
    assert np.all(rel <= gam), rel


@pytest.mark.parametrize("which", [1, 2])
def test_probes_compute_rowsum_times_x(which):
    # both probes give y_i = x_min(i, n_cols-1) * sum_j a_ij (dyadic: exact)
    for n, m, rp, col, val in (synth.tiny_random(400, 300, 0.05, 9, dyadic=True),
                               synth.tiny_random(200, 450, 0.1, 10, dyadic=True)):
        x = synth.dyadic_vector(m, 11)
        A = pkg.CsrMatrix(rp, col, val, n_cols=m)
        y = A.probe(which, torch.from_numpy(x).cuda())
        torch.cuda.synchronize()
        rows = np.repeat(np.arange(n), np.diff(rp))
        ref = oracle.spmv(rp, np.minimum(rows, m - 1).astype(np.int32), val, x)
        assert np.array_equal(y.cpu().numpy(), ref)


def long_rows_matrix(seed=5):
    lens = [0, 0, 5000, 1, 0, 30000, 0, 0, 2, 100000, 0] + [3] * 500 + [0] * 100 + [9000]
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    col = np.concatenate([np.sort(synth.uindex(seed, i, np.arange(l, dtype=np.uint64), 200000))
                          for i, l in enumerate(lens)]).astype(np.int32)
    return len(lens), 200000, rp, col


@pytest.mark.parametrize("extra", [0, pkg.OPT_PREFETCH, pkg.OPT_UNROLL, pkg.OPT_DELTA])
def test_decomposition(extra):
    n, m, rp, col = long_rows_matrix()
    # distinct sorted columns are required by delta codes: deduplicate rows
    keep = np.ones(len(col), dtype=bool)
    for i in range(n):
        seg = col[rp[i]:rp[i + 1]]
        keep[rp[i] + 1:rp[i + 1]] = seg[1:] != seg[:-1]
    rows = np.repeat(np.arange(n), np.diff(rp))[keep]
    _, _, rp, col, _ = synth.from_coo(rows, col[keep], np.zeros(keep.sum()), n, m)
    val = (synth.uindex(6, 0, np.arange(len(col), dtype=np.uint64), 9) - 4).astype(float)
    x = synth.dyadic_vector(m, 12)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    info = A.select("forced", forced_opts=pkg.OPT_DECOMP | extra, long_row_floor=1000,
                    long_row_factor=4.0)
    tau = oracle.long_row_threshold(len(col) / n, factor=4.0, floor=1000)
    want_rows = oracle.long_rows(rp, tau)
    assert info["n_long_rows"] == len(want_rows) > 0
    assert np.array_equal(A.debug_copy(pkg.DEBUG_LONG_ROWS, np.int32), want_rows)
    xd = torch.from_numpy(x).cuda()
    y = A.spmv(xd)
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), oracle.spmv(rp, col, val, x))   # dyadic: exact
    vr = synth.um11(7, 0, np.arange(len(col), dtype=np.uint64))
    B = pkg.CsrMatrix(rp, col, vr, n_cols=m)
    B.select("forced", forced_opts=pkg.OPT_DECOMP | extra, long_row_floor=1000, long_row_factor=4.0)
    xr = synth.vector(m, 13)
    y = B.spmv(torch.from_numpy(xr).cuda())
    torch.cuda.synchronize()
    check_f64(y.cpu().numpy(), rp, col, vr, xr, f"decomp {extra}")


def test_decomposition_rmat():
    n, m, rp, col, val = matrix("rmat14")
    x = xvec("rmat14", m)
    A = pkg.CsrMatrix(rp, col, val)
    info = A.select("forced", forced_opts=pkg.OPT_DECOMP, long_row_floor=200, long_row_factor=8.0)
    assert info["n_long_rows"] > 0
    y = A.spmv(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    check_f64(y.cpu().numpy(), rp, col, val, x, "rmat14 decomp")


def check_tables_in_place(A, info, rp):
    """The autotuner rebuilds the merge tile table per candidate tile size;
    the one left in place must be the table of the plan it kept."""
    if info["opts"] & pkg.OPT_MERGE:
        ti, tj = oracle.merge_tiles(rp, info["merge_items"], info["merge_slack"])
        assert np.array_equal(A.debug_copy(pkg.DEBUG_TILE_I, np.int32), ti)
        assert np.array_equal(A.debug_copy(pkg.DEBUG_TILE_J, np.int32), tj)


@pytest.mark.parametrize("name", ["lap100", "st27_24", "rmat14", "unif14"])
def test_profile_rule_and_remedies_match_oracle(name):
    n, m, rp, col, val = matrix(name)
    A = pkg.CsrMatrix(rp, col, val)
    info = A.select("profile")
    p = info
    assert p["p_peak"] >= p["p_mb"] > 0 and p["p_csr"] > 0 and p["b_max"] > 1e11
    d = pkg.default_config()
    cls = oracle.classify(p["p_csr"], p["p_mb"], p["p_ml"], p["p_imb"], p["p_cmp"], p["p_peak"],
                          t_ml=d.t_ml, t_imb=d.t_imb, t_mb=d.t_mb)
    assert info["classes"] == cls
    f, _ = oracle.features(n, m, rp, col)
    has_long = f[F["nnz_max"]] > oracle.long_row_threshold(f[F["nnz_avg"]])
    assert info["opts"] == oracle.remedies(cls, has_long, d.remedy_map)
    check_tables_in_place(A, info, rp)
    x = xvec(name, m)
    y = A.spmv(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    check_f64(y.cpu().numpy(), rp, col, val, x, f"{name} profile")


@pytest.mark.parametrize("name,storage", [("lap100", "f64"), ("unif14", "f64"),
                                          ("rmat14", "f32"), ("st27_24", "bf16")])
def test_profile_bounds_match_oracle_formulas(name, storage):
    # Sec. III-B: P_MB and P_peak from B_max and the compulsory bytes, P_IMB
    # = 2 NNZ / t_median over the per-CU spans; B_max is the cache triad's
    # figure when the working set fits in the 256 MB Infinity Cache
    n, m, rp, col, val = matrix(name)
    A = pkg.CsrMatrix(rp, col, val, storage=storage)
    info = A.select("profile")
    nnz = len(col)
    b_hbm, b_cache, clock_hz = A.debug_copy(pkg.DEBUG_BANDWIDTH, np.float64)
    assert (b_hbm, b_cache) == pkg.device_bandwidth()
    vb = {"f64": 8, "f32": 4, "bf16": 2}[storage]
    xb = 8 if storage == "f64" else 4
    s_fmt = oracle.format_bytes(n, m, nnz, val_bytes=vb)
    s_x, s_y = xb * m, xb * n
    b_max = oracle.b_for_footprint(s_fmt + s_x + s_y, b_hbm, b_cache)
    assert info["b_max"] == b_max
    assert info["p_mb"] == oracle.p_mb(nnz, s_fmt, s_x, s_y, b_max)
    assert info["p_peak"] == oracle.p_peak(nnz, vb * nnz, s_x, s_y, b_max)
    spans = A.debug_copy(pkg.DEBUG_IMB_SPANS, np.int64)
    assert 1 <= spans.size <= 256 and np.all(spans > 0)
    assert clock_hz > 0
    assert info["p_imb"] == pytest.approx(oracle.p_imb(nnz, spans / clock_hz), rel=1e-14)
    d = pkg.default_config()
    cls = oracle.classify(info["p_csr"], info["p_mb"], info["p_ml"], info["p_imb"],
                          info["p_cmp"], info["p_peak"], t_ml=d.t_ml, t_imb=d.t_imb, t_mb=d.t_mb)
    assert info["classes"] == cls


@pytest.mark.parametrize("streaming", [True, False])
def test_triad_kernel_output(streaming):
    # dyadic b, c and s = 3: every b + s c is exact, so the FMA's one
    # rounding gives the exact value
    n = (1 << 20) + 2
    b = synth.dyadic_vector(n, 41)
    c = synth.dyadic_vector(n, 42)
    bd, cd = torch.from_numpy(b).cuda(), torch.from_numpy(c).cuda()
    ad = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
    pkg.debug_triad(ad, bd, cd, 3.0, streaming)
    torch.cuda.synchronize()
    assert np.array_equal(ad.cpu().numpy(), b + 3.0 * c)


def test_device_bandwidth_pair():
    hbm, cache = pkg.device_bandwidth()
    assert 1e12 < hbm < 9e12
    assert cache >= hbm


def test_exhaustive_selects_catalogue_variant():
    n, m, rp, col, val = matrix("st27_24")
    A = pkg.CsrMatrix(rp, col, val)
    info = A.select("exhaustive", timing_calls=8)
    assert 0 <= info["variant_id"] < 16
    assert oracle.catalogue()[info["variant_id"]] == info["opts"]
    check_tables_in_place(A, info, rp)
    x = xvec("st27_24", m)
    y = A.spmv(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    check_f64(y.cpu().numpy(), rp, col, val, x, "exhaustive")


def test_exhaustive_single_remedies_only():
    """exhaustive_set = 1 (the trivial-single optimizer of Sec. IV-D) keeps
    the fastest of the baseline and the 5 single remedies; other values are
    rejected."""
    n, m, rp, col, val = matrix("rmat14")
    A = pkg.CsrMatrix(rp, col, val)
    info = A.select("exhaustive", timing_calls=8, exhaustive_set=1)
    assert 0 <= info["variant_id"] <= 5
    assert info["opts"] in (0, 1, 2, 4, 8, 16)
    check_tables_in_place(A, info, rp)
    x = xvec("rmat14", m)
    y = A.spmv(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    check_f64(y.cpu().numpy(), rp, col, val, x, "exhaustive singles")
    with pytest.raises(pkg.CsrError):
        A.select("exhaustive", exhaustive_set=2)


def test_every_catalogue_variant_matches_oracle():
    n, m, rp, col, val = matrix("rmat14")
    x = xvec("rmat14", m)
    A = pkg.CsrMatrix(rp, col, val)
    for opts in oracle.catalogue():
        A.select("forced", forced_opts=opts, long_row_floor=200)
        y = A.spmv(torch.from_numpy(x).cuda())
        torch.cuda.synchronize()
        check_f64(y.cpu().numpy(), rp, col, val, x, f"catalogue {opts}")


def partition_rows_per_block(n, nblk):
    ng = [g for g in (4, 8, 16, 32, 64, 128, 256) if -(-n // g) == nblk]
    assert len(ng) == 1, (n, nblk, ng)
    return ng[0]


def check_partition_records(A, n, rp, Q, t_part):
    """Bounds bit-exact against the oracle's nnz-balanced partitioning, the
    ratios exactly the oracle's from the recorded block times, and the plan
    info's summary consistent with them."""
    bounds = A.debug_copy(pkg.DEBUG_MLP_BOUNDS, np.int32)
    times = A.debug_copy(pkg.DEBUG_MLP_TIMES, np.int64)
    ratios = A.debug_copy(pkg.DEBUG_MLP_RATIOS, np.float64)
    nblk = times.size // 2
    NG = partition_rows_per_block(n, nblk)
    np.testing.assert_array_equal(bounds, oracle.ml_partition_bounds(rp, NG, Q))
    assert (times >= 0).all()
    ref = oracle.ml_partition_ratios(times[:nblk], times[nblk:], bounds)
    np.testing.assert_array_equal(ratios, ref)
    info = A.info
    assert info["ml_partitions"] == int((ratios > 0).sum())
    assert info["ml_parts_flagged"] == int((ratios > t_part).sum())
    assert info["ml_part_max"] == ratios.max()
    return bounds, ratios, NG


def test_partition_aware_ml_finds_a_local_irregular_stretch():
    """1/64 of the rows gather at random columns, the rest are banded: the
    flagged partitions all overlap the irregular stretch, ML is set, and the
    largest partition ratio exceeds the whole-matrix P_ML / P_CSR."""
    n, m, rp, col, val = synth.localized_irregular(1 << 21, 16, 1 / 64, 811)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    info = A.select("profile", ml_partitions=256, autotune=0)
    bounds, ratios, NG = check_partition_records(A, n, rp, 256, 1.5)
    r0, r1 = n // 2, n // 2 + round(n / 64)
    flagged = np.nonzero(ratios > 1.5)[0]
    assert flagged.size > 0, ratios.max()
    for q in flagged:
        lo, hi = bounds[q] * NG, min(bounds[q + 1] * NG, n)
        assert lo < r1 and hi > r0, (q, lo, hi)
    assert info["classes"] & oracle.CLS_ML
    assert info["ml_part_max"] > info["p_ml"] / info["p_csr"]
    y = A.spmv(torch.from_numpy(synth.vector(m, 3)).cuda())
    check_f64(y.cpu().numpy(), rp, col, val, synth.vector(m, 3), "localized irregular")
    A.close()


def test_partition_aware_ml_quiet_on_banded_rows():
    n, m, rp, col, val = synth.localized_irregular(1 << 21, 16, 0.0, 811)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    info = A.select("profile", ml_partitions=256, autotune=0)
    check_partition_records(A, n, rp, 256, 1.5)
    assert info["ml_parts_flagged"] == 0 and info["ml_part_max"] < 1.5
    # off by default: no records, and the plan info says so
    info = A.select("profile", autotune=0)
    assert info["ml_partitions"] == 0 and info["ml_part_max"] == 0.0
    with pytest.raises(pkg.CsrError):
        A.debug_copy(pkg.DEBUG_MLP_BOUNDS, np.int32)
    A.close()


@pytest.mark.parametrize("Q", [1, 7, 4096])
def test_partition_records_small_and_ragged(Q):
    """More partitions than row blocks (empty partitions), a single one, and
    a ragged last block with empty rows."""
    n, m, rp, col, val = unsorted_with_empty_rows()
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    A.select("profile", ml_partitions=Q, t_ml_part=2.0, autotune=0)
    check_partition_records(A, n, rp, Q, 2.0)
    A.close()


def test_partition_config_rejected():
    n, m, rp, col, val = feature_case("tiny")
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    for bad in ({"ml_partitions": 4097}, {"ml_partitions": -1},
                {"ml_partitions": 8, "t_ml_part": 0.0}):
        with pytest.raises(pkg.CsrError):
            A.select("profile", **bad)
    A.close()

"""Pins of the oracle's matrix features (Sec. III-D, Table I): closed forms of
the 2-D Laplacian derived by hand, the 27-point row-length histogram, and a
brute-force per-row recomputation with Python sets on small random matrices."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
F = {name: k for k, name in enumerate(oracle.FEATURE_NAMES)}
I = {name: k for k, name in enumerate(oracle.FEATURE_INT_NAMES)}


def test_laplacian_closed_forms():
    g = json.load(open(os.path.join(GOLDEN, "laplacian100_features.json")))
    n, m, rp, col, _ = synth.laplacian2d(100)
    f, s = oracle.features(n, m, rp, col)
    assert f[F["N"]] == g["N"]
    assert f[F["nnz_min"]] == g["nnz_min"] and f[F["nnz_max"]] == g["nnz_max"]
    assert s[I["sum_nnz"]] == g["sum_nnz"] and s[I["sum_nnz2"]] == g["sum_nnz2"]
    assert s[I["sum_bw"]] == g["sum_bw"] and s[I["sum_bw2"]] == g["sum_bw2"]
    assert s[I["sum_misses"]] == g["sum_misses"] and s[I["sum_groups"]] == g["sum_groups"]
    assert f[F["bw_min"]] == g["bw_min"] and f[F["bw_max"]] == g["bw_max"]
    assert math.isclose(f[F["nnz_avg"]], 4.96, rel_tol=1e-15)
    assert math.isclose(f[F["nnz_sd"]], math.sqrt(g["nnz_var"]), rel_tol=1e-12)
    assert math.isclose(f[F["bw_avg"]], 198.0198, rel_tol=1e-15)
    assert math.isclose(f[F["bw_sd"]], math.sqrt(g["bw_var"]), rel_tol=1e-12)
    assert math.isclose(f[F["misses_avg"]], 2.98, rel_tol=1e-15)
    # FP sums over N = 10^4 rows carry at most gamma_N = N u / (1 - N u)
    # relative rounding error (all terms are positive)
    gam = 1e4 * 2.0 ** -53 / (1 - 1e4 * 2.0 ** -53) + 2.0 ** -52
    clus = (9604 * 0.6 + 98 + 147 + 8 / 3) / 10000
    assert math.isclose(f[F["clustering_avg"]], clus, rel_tol=gam)
    terms = g["scatter_terms"]
    sc_avg = sum(c * a / b for c, a, b in terms) / 10000
    sc_var = sum(c * (a / b - sc_avg) ** 2 for c, a, b in terms) / 10000
    assert math.isclose(f[F["scatter_avg"]], sc_avg, rel_tol=gam)
    assert math.isclose(f[F["scatter_sd"]], math.sqrt(sc_var), rel_tol=1e-10)
    assert math.isclose(f[F["mean_col_gap"]], 1980198 / 39600, rel_tol=1e-15)
    assert f[F["size"]] == g["size"]


def test_stencil27_row_length_histogram():
    n, m, rp, col, _ = synth.stencil27(128)
    f, s = oracle.features(n, m, rp, col)
    # 126^3 interior rows with 27, 6*126^2 face rows with 18, 12*126 edge rows
    # with 12, 8 corners with 8 entries
    hist = {27: 126 ** 3, 18: 6 * 126 ** 2, 12: 12 * 126, 8: 8}
    assert hist == {27: 2000376, 18: 95256, 12: 1512, 8: 8}
    assert s[I["sum_nnz"]] == sum(k * c for k, c in hist.items())
    assert s[I["sum_nnz2"]] == sum(k * k * c for k, c in hist.items())
    assert f[F["nnz_min"]] == 8 and f[F["nnz_max"]] == 27
    assert f[F["size"]] == 0.0  # 710.9 MB does not fit a 256 MiB cache


def _brute(n_rows, n_cols, rp, col):
    nnz = [rp[i + 1] - rp[i] for i in range(n_rows)]
    bw, sc, cl, miss, grp = [], [], [], [], []
    for i in range(n_rows):
        c = [int(v) for v in col[rp[i]:rp[i + 1]]]
        if not c:
            bw.append(0), sc.append(0.0), cl.append(0.0), miss.append(0), grp.append(0)
            continue
        b = max(c) - min(c)
        runs = 1 + sum(1 for a, bb in zip(c, c[1:]) if bb != a + 1)
        ms = 1 + sum(1 for a, bb in zip(c, c[1:]) if abs(bb - a) > 16)
        bw.append(b), sc.append(len(c) / max(b, 1)), cl.append(runs / len(c))
        miss.append(ms), grp.append(runs)
    N = n_rows
    shared = distinct = 0
    if N > 1:
        S = min(4096, N - 1)
        for s in range(S):
            r = 1 + (s * (N - 1)) // S
            cur = [int(v) >> 4 for v in col[rp[r]:rp[r + 1]][:256]]
            prev = set(int(v) >> 4 for v in col[rp[r - 1]:rp[r]][:256])
            heads = [v for k, v in enumerate(cur) if k == 0 or cur[k - 1] != v]
            distinct += len(heads)
            shared += sum(1 for v in heads if v in prev)
    pstd = lambda a: float(np.std(np.asarray(a, dtype=np.float64))) if a else 0.0
    mean = lambda a: float(np.mean(np.asarray(a, dtype=np.float64))) if a else 0.0
    tot1 = sum(max(k - 1, 0) for k in nnz)
    return {
        "nnz_min": min(nnz), "nnz_max": max(nnz), "nnz_avg": mean(nnz), "nnz_sd": pstd(nnz),
        "bw_min": min(bw), "bw_max": max(bw), "bw_avg": mean(bw), "bw_sd": pstd(bw),
        "scatter_avg": mean(sc), "scatter_sd": pstd(sc), "clustering_avg": mean(cl),
        "misses_avg": mean(miss), "mean_col_gap": (sum(bw) / tot1) if tot1 else 0.0,
        "x_reuse": shared / distinct if distinct else 0.0,
        "_int": [sum(nnz), sum(k * k for k in nnz), sum(bw), sum(b * b for b in bw), sum(miss),
                 sum(grp), shared, distinct],
    }


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_small(seed):
    if seed == 5:
        # unsorted rows with duplicates: features are defined in storage order
        m, n = 50, 70
        rp = np.arange(0, 501, 10, dtype=np.int32)
        col = synth.uindex(9, 0, np.arange(500, dtype=np.uint64), n).astype(np.int32)
    else:
        m, n, rp, col, _ = synth.tiny_random(60 + 40 * seed, 90 + 300 * seed, 0.02 + 0.05 * seed, seed)
    f, s = oracle.features(m, n, rp, col)
    b = _brute(m, n, rp, col)
    assert list(s) == b["_int"]
    for name, v in b.items():
        if name == "_int":
            continue
        assert math.isclose(f[F[name]], v, rel_tol=1e-12, abs_tol=1e-14), name


def test_x_reuse_extremes():
    # every row identical -> all lines shared; disjoint far-apart rows -> none
    n = 300
    rp = np.arange(0, 4 * n + 1, 4, dtype=np.int32)
    same = np.tile(np.array([0, 16, 32, 48], dtype=np.int32), n)
    f, _ = oracle.features(n, 1000, rp, same)
    assert f[F["x_reuse"]] == 1.0
    far = (np.arange(4 * n, dtype=np.int64) * 64).astype(np.int32)
    f, _ = oracle.features(n, 64 * 4 * n, rp, far)
    assert f[F["x_reuse"]] == 0.0


def test_empty_and_single_row():
    f, s = oracle.features(0, 0, np.array([0], dtype=np.int32), np.zeros(0, dtype=np.int32))
    assert np.all(f[:13] == 0) and np.all(s == 0)
    f, s = oracle.features(1, 10, np.array([0, 3], dtype=np.int32), np.array([2, 3, 9], dtype=np.int32))
    assert f[F["bw_max"]] == 7 and f[F["x_reuse"]] == 0.0 and s[I["sum_groups"]] == 2

"""Shared helpers for the GPU parity tests: cached seeded matrices, the
oracle's reference and error scale, and the comparison bars.

FP64 bar (per row): |y - y_acc| <= 1e-12 * (|A||x|)_i, where y_acc is the
oracle's compensated (Dot2) product, and rows with |A||x| = 0 must be exactly
zero. FP32/BF16 storage: |y - y_q| <= gamma_{n_i+1}(2^-24) * (|A_q||x_q|)_i
against the accurate product of the stored values (any FP32 summation order
satisfies it)."""
from __future__ import annotations

import functools

import numpy as np

import oracle
import synth


@functools.lru_cache(maxsize=None)
def matrix(name: str):
    if name == "lap100":
        return synth.laplacian2d(100)
    if name == "lap37":
        return synth.laplacian2d(37, 23)
    if name == "st27_128":
        return synth.stencil27(128)
    if name == "st27_24":
        return synth.stencil27(24)
    if name == "rmat22":
        return synth.rmat(22)
    if name == "rmat22perm":
        return permuted(*matrix("rmat22"), seed=304)
    if name == "rmat14":
        return synth.rmat(14, 16)
    if name == "unif20":
        return synth.uniform_random(1 << 20, 16)
    if name == "unif14":
        return synth.uniform_random(1 << 14, 16)
    if name == "unif17":
        return synth.uniform_random(1 << 17, 16)
    if name == "unif600k":  # x of 4.8 MB: more than one XCD's L2
        return synth.uniform_random(600_000, 8)
    raise KeyError(name)


def permuted(n, m, rp, col, val, seed):
    """Symmetric permutation P A P^T with the seeded Fisher-Yates permutation p
    (row i moves to p[i], column j to p[j]), rows sorted by column."""
    p = synth.permutation(n, seed).astype(np.int64)
    inv = np.empty_like(p)
    inv[p] = np.arange(n)
    lens = np.diff(rp).astype(np.int64)[inv]           # new row r is old row inv[r]
    nrp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=nrp[1:])
    src = np.repeat(rp[:-1].astype(np.int64)[inv] - nrp[:-1], lens) + np.arange(nrp[-1])
    rows = np.repeat(np.arange(n, dtype=np.int64), lens)
    cols = p[col[src]]
    order = np.argsort(rows * m + cols, kind="stable")
    return n, m, nrp.astype(np.int32), cols[order].astype(np.int32), val[src][order]


X_SEED = {"lap100": 101, "st27_128": 203, "rmat22": 303, "rmat22perm": 303, "unif20": 403}


def xvec(name: str, n: int):
    return synth.vector(n, X_SEED.get(name, 999))


def check_f64(y, rp, col, val, x, what=""):
    y = np.asarray(y, dtype=np.float64)
    ref = oracle.spmv_accurate(rp, col, val, x)
    ab = oracle.absax(rp, col, val, x)
    err = np.abs(y - ref)
    bad = ~(err <= 1e-12 * ab)
    if bad.any():
        i = int(np.nonzero(bad)[0][0])
        raise AssertionError(f"{what}: {int(bad.sum())} rows off; first row {i}: "
                             f"y={y[i]!r} ref={ref[i]!r} |A||x|={ab[i]!r}")


def check_reduced(y, rp, col, val, x, storage, what=""):
    yq, bound = oracle.reduced_precision_bound(rp, col, val, x, storage)
    err = np.abs(np.asarray(y, dtype=np.float64) - yq)
    bad = ~(err <= bound)
    if bad.any():
        i = int(np.nonzero(bad)[0][0])
        raise AssertionError(f"{what}: {int(bad.sum())} rows off; row {i}: y={y[i]!r} "
                             f"ref={yq[i]!r} bound={bound[i]!r}")
    return oracle.rel_error_report(y, oracle.spmv_accurate(rp, col, val, x),
                                   oracle.absax(rp, col, val, x))

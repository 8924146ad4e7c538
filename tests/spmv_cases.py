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


X_SEED = {"lap100": 101, "st27_128": 203, "rmat22": 303, "unif20": 403}


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

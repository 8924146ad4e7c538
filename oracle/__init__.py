"""CPU oracle for the adaptive CSR SpMV method (Elafrou, Goumas & Koziris 2017).

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package. The GPU library never
calls it, and it shares no code with the GPU library (`paper_1711_05487_amd`).

Two parts:

* ``csr_oracle.c`` (plain C, ``gcc -O2 -ffp-contract=off``), loaded with ctypes:
  SpMV in storage order, |A||x|, the Dot2 accurate reference, dense matvec,
  CSR validation, FP32/BF16 rounding, delta codes, merge-path tiles, long-row
  list and the matrix features.
* Pure Python/numpy here: the per-class bounds, the profile-guided rule, the
  class-to-optimization map, the amortization count, the reduced-precision
  error report, feature normalization and the FP64 MLP with its gradients and
  Adam.

Every function cites the part of the paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

GCC_FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = False) -> str:
    """Compile csr_oracle.c into liboracle.so with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, c_int = ctypes.c_int32, ctypes.c_int64, ctypes.c_int
        sig = {
            "or_spmv": (None, [i32, P, P, P, P, P]),
            "or_absax": (None, [i32, P, P, P, P, P]),
            "or_spmv_dot2": (None, [i32, P, P, P, P, P]),
            "or_dense_matvec": (None, [i32, i32, P, P, P]),
            "or_csr_valid": (c_int, [i32, i32, i64, P, P]),
            "or_rows_sorted": (c_int, [i32, P, P]),
            "or_to_f32": (None, [i64, P, P]),
            "or_to_bf16": (None, [i64, P, P]),
            "or_bf16_to_f64": (None, [i64, P, P]),
            "or_delta_eligible": (c_int, [i32, P, P, c_int]),
            "or_delta_encode": (c_int, [i32, P, P, c_int, P]),
            "or_delta_decode": (None, [i32, P, P, c_int, P]),
            "or_merge_tiles": (i64, [i32, P, i64, i64, P, P]),
            "or_merge_codes": (c_int, [i64, P, P, c_int, P, P]),
            "or_window_codes": (c_int, [i64, P, P, c_int, P, P, P, P]),
            "or_column_blocks": (None, [i32, P, P, P, i32, i32, P, P, P]),
            "or_long_rows": (i32, [i32, P, i64, P]),
            "or_features": (None, [i32, i32, P, P, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr(rp, col):
    return (np.ascontiguousarray(rp, dtype=np.int32), np.ascontiguousarray(col, dtype=np.int32))


# ---------------------------------------------------------------------------
# SpMV and its error scale (Sec. II, Fig. 2)
# ---------------------------------------------------------------------------

def spmv(rp, col, val, x) -> np.ndarray:
    """y = A x, each row summed from +0.0 in storage order (Sec. II, Fig. 2)."""
    rp, col = _csr(rp, col)
    val = np.ascontiguousarray(val, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(rp.size - 1, dtype=np.float64)
    lib().or_spmv(rp.size - 1, _p(rp), _p(col), _p(val), _p(x), _p(y))
    return y


def absax(rp, col, val, x) -> np.ndarray:
    """Per-row sum of |a_ij| |x_j|."""
    rp, col = _csr(rp, col)
    val = np.ascontiguousarray(val, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(rp.size - 1, dtype=np.float64)
    lib().or_absax(rp.size - 1, _p(rp), _p(col), _p(val), _p(x), _p(y))
    return y


def spmv_accurate(rp, col, val, x) -> np.ndarray:
    """y = A x by compensated dot products (Ogita-Rump-Oishi Dot2)."""
    rp, col = _csr(rp, col)
    val = np.ascontiguousarray(val, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(rp.size - 1, dtype=np.float64)
    lib().or_spmv_dot2(rp.size - 1, _p(rp), _p(col), _p(val), _p(x), _p(y))
    return y


def dense_matvec(a, x) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(a.shape[0], dtype=np.float64)
    lib().or_dense_matvec(a.shape[0], a.shape[1], _p(a), _p(x), _p(y))
    return y


def csr_valid(n_rows, n_cols, nnz, rp, col) -> bool:
    rp, col = _csr(rp, col)
    if rp.size != n_rows + 1:
        return False
    if col.size < nnz:
        return False
    return bool(lib().or_csr_valid(n_rows, n_cols, nnz, _p(rp), _p(col)))


def rows_sorted(rp, col) -> bool:
    rp, col = _csr(rp, col)
    return bool(lib().or_rows_sorted(rp.size - 1, _p(rp), _p(col)))


# ---------------------------------------------------------------------------
# Reduced-precision value storage
# ---------------------------------------------------------------------------

def to_f32(v) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.empty(v.size, dtype=np.float32)
    lib().or_to_f32(v.size, _p(v), _p(out))
    return out


def to_bf16_bits(v) -> np.ndarray:
    """FP64 -> BF16 bit patterns (uint16), one round-to-nearest-even step."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.empty(v.size, dtype=np.uint16)
    lib().or_to_bf16(v.size, _p(v), _p(out))
    return out


def bf16_bits_to_f64(b) -> np.ndarray:
    b = np.ascontiguousarray(b, dtype=np.uint16)
    out = np.empty(b.size, dtype=np.float64)
    lib().or_bf16_to_f64(b.size, _p(b), _p(out))
    return out


def quantize(v, storage: str) -> np.ndarray:
    """The FP64 value of each stored element for storage 'f64'|'f32'|'bf16'."""
    if storage == "f64":
        return np.asarray(v, dtype=np.float64)
    if storage == "f32":
        return to_f32(v).astype(np.float64)
    if storage == "bf16":
        return bf16_bits_to_f64(to_bf16_bits(v))
    raise ValueError(storage)


# Unit roundoff of each storage format: 2^-p for p significand bits.
UNIT_ROUNDOFF = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "bf16": 2.0 ** -8}


def reduced_precision_bound(rp, col, val, x, storage: str):
    """Reference and a-priori error bound for FP32-accumulated SpMV with values
    and x stored in `storage` (x rounded once to FP32 for f32/bf16 stores).

    Returns (y_q, bound): y_q is the accurate product of the *stored* values
    and the FP32 x; bound_i = gamma_{n_i+1}(2^-24) * sum |v_q| |x_q| bounds the
    error of any FP32 summation order of the row's n_i rounded products."""
    vq = quantize(val, storage)
    xq = to_f32(x).astype(np.float64)
    yq = spmv_accurate(rp, col, vq, xq)
    ab = absax(rp, col, vq, xq)
    n = np.diff(np.asarray(rp, dtype=np.int64)).astype(np.float64)
    u = 2.0 ** -24
    k = n + 1.0
    gamma = np.where(k * u < 1.0, (k * u) / np.maximum(1.0 - k * u, 1e-300), np.inf)
    return yq, gamma * ab


def rel_error_report(y, y_ref, ab) -> dict:
    """Per-row relative error |y - y_ref| / (|A||x|), normalized by |A||x| so a
    cancelled y_ref does not blow up the ratio; rows with |A||x| = 0 must be 0."""
    y = np.asarray(y, dtype=np.float64)
    d = np.abs(y - y_ref)
    nz = ab > 0
    rel = np.zeros_like(d)
    rel[nz] = d[nz] / ab[nz]
    bad_zero = bool((d[~nz] != 0).any())
    return {"max": float(rel.max(initial=0.0)),
            "p99": float(np.percentile(rel, 99)) if rel.size else 0.0,
            "zero_rows_exact": not bad_zero}


# ---------------------------------------------------------------------------
# MB remedy: delta-encoded column indices (Sec. III-E, Table II)
# ---------------------------------------------------------------------------

def delta_eligible(rp, col, w: int) -> bool:
    rp, col = _csr(rp, col)
    return bool(lib().or_delta_eligible(rp.size - 1, _p(rp), _p(col), w))


def delta_encode(rp, col, w: int):
    """w-bit codes (uint8/uint16 array) or None if the matrix is not eligible."""
    rp, col = _csr(rp, col)
    out = np.empty(col.size, dtype=np.uint8 if w == 8 else np.uint16)
    ok = lib().or_delta_encode(rp.size - 1, _p(rp), _p(col), w, _p(out))
    return out if ok else None


def delta_decode(rp, codes, w: int) -> np.ndarray:
    rp = np.ascontiguousarray(rp, dtype=np.int32)
    codes = np.ascontiguousarray(codes, dtype=np.uint8 if w == 8 else np.uint16)
    col = np.empty(codes.size, dtype=np.int32)
    lib().or_delta_decode(rp.size - 1, _p(rp), _p(codes), w, _p(col))
    return col


def delta_width(rp, col) -> int:
    """Smallest eligible width (8, then 16), or 32 when neither fits."""
    for w in (8, 16):
        if delta_eligible(rp, col, w):
            return w
    return 32


# ---------------------------------------------------------------------------
# IMB remedies (Sec. III-E): merge-path tiles and long-row decomposition
# ---------------------------------------------------------------------------

def merge_codes(tj, col, w: int):
    """Tile-base column codes of the merge path (MB remedy, Table II): per
    tile the smallest column, per nonzero the w-bit offset from it; None when
    some tile's column range does not fit in w bits."""
    tj = np.ascontiguousarray(tj, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    T = tj.size - 1
    base = np.zeros(max(T, 1), dtype=np.int32)
    codes = np.zeros(max(col.size, 1), dtype=np.uint16 if w == 16 else np.uint8)
    if not lib().or_merge_codes(T, _p(tj), _p(col), w, _p(base), codes.ctypes.data_as(ctypes.c_void_p)):
        return None
    return base[:T], codes[:col.size]


def window_codes(tj, col, maxw: int = 256):
    """Window codes of row-aligned merge tiles (MB + ML remedies, Table II):
    per tile t the ascending distinct columns u_0 < ... < u_{m-1}, stored as
    base_t = u_0 and dict[t, k] = u_k - u_0; per nonzero the rank of its
    column in the window. Returns (base, wlen, dict, codes) with dict of
    shape (T, maxw), zero past wlen, and codes uint8 (maxw <= 256) or the
    full uint16 ranks (windows of up to 512 entries); None when some tile
    has more than maxw distinct columns or a column range of 2^16 or more."""
    tj = np.ascontiguousarray(tj, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    T = tj.size - 1
    base = np.zeros(max(T, 1), dtype=np.int32)
    wlen = np.zeros(max(T, 1), dtype=np.int32)
    dct = np.zeros((max(T, 1), maxw), dtype=np.uint16)
    codes = np.zeros(max(col.size, 1), dtype=np.uint16)
    if not lib().or_window_codes(T, _p(tj), _p(col), maxw, _p(base), _p(wlen),
                                 dct.ctypes.data_as(ctypes.c_void_p),
                                 codes.ctypes.data_as(ctypes.c_void_p)):
        return None
    codes = codes[:col.size]
    return base[:T], wlen[:T], dct[:T], codes.astype(np.uint8) if maxw <= 256 else codes


def window_rank_records(tj, ranks, wlen, vec: int, lanes: int = 64):
    """Where 9-bit window ranks keep their ninth bit: per tile a record of
    1 + lanes / 2 int32 words, [0] = the window length, then lanes 16-bit
    masks (two per word, the lower lane in the low half). Lane l's mask has
    bit it * vec + e set when the rank of tile element it * lanes * vec +
    l * vec + e (the element that lane loads as entry e of its load block
    it) is 256 or more."""
    tj = np.asarray(tj, dtype=np.int64)
    ranks = np.asarray(ranks, dtype=np.int64)
    T = tj.size - 1
    masks = np.zeros((max(T, 0), lanes), dtype=np.int64)
    for t in range(T):
        for p in range(int(tj[t + 1] - tj[t])):
            if ranks[tj[t] + p] >= 256:
                it, r = divmod(p, lanes * vec)
                lane, e = divmod(r, vec)
                masks[t, lane] |= 1 << (it * vec + e)
    rec = np.zeros((max(T, 0), 1 + lanes // 2), dtype=np.int64)
    rec[:, 0] = np.asarray(wlen, dtype=np.int64)[:T]
    rec[:, 1:] = masks[:, 0::2] | (masks[:, 1::2] << 16)
    return rec.astype(np.uint32).view(np.int32)


def window_runs(tj, col, max_runs: int = 14):
    """Run windows of row-aligned merge tiles (MB + ML remedies, Table II):
    the window of a tile (its distinct columns, ascending: u_0 < ... < u_{m-1},
    at most 256 of them within a range below 2^16) written as maximal runs of
    consecutive columns. Per tile a record of 16 int32 words: [0] = u_0 (0
    for a tile without nonzeros), [1] = m | (number of runs << 16), [2 + r] =
    (first column of run r - u_0) | (length of run r << 16), zero past the
    last run; per nonzero the 8-bit rank of its column in the window (as for
    window codes). Returns (records of shape (T, 16), codes), or None when
    some tile has more than max_runs runs, more than 256 distinct columns or
    a range of 2^16 or more."""
    assert 1 <= max_runs <= 14, "a record holds at most 14 runs"
    tj = np.asarray(tj, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    T = tj.size - 1
    rec = np.zeros((max(T, 0), 16), dtype=np.int64)
    codes = np.zeros(col.size, dtype=np.uint8)
    for t in range(T):
        c = col[tj[t]:tj[t + 1]]
        if c.size == 0:
            continue
        u = np.unique(c)
        if u.size > 256 or u[-1] - u[0] >= 65536:
            return None
        # a run starts at the first column and wherever the next column is
        # not the previous one plus one
        starts = [0] + [k for k in range(1, u.size) if u[k] != u[k - 1] + 1]
        if len(starts) > max_runs:
            return None
        ends = starts[1:] + [u.size]
        rec[t, 0] = u[0]
        rec[t, 1] = u.size | (len(starts) << 16)
        for r, (a, b) in enumerate(zip(starts, ends)):
            rec[t, 2 + r] = (u[a] - u[0]) | ((b - a) << 16)
        codes[tj[t]:tj[t + 1]] = np.searchsorted(u, c)
    return rec.astype(np.int32), codes


def merge_tiles(rp, L: int, slack: int = 0):
    """(i_t, j_t) for t = 0..T of the merge path of the row ends with the
    nonzeros, cut every L items; with slack s > 0 cut every L - s items and
    move each cut forward to the end of the row in progress (row-aligned
    tiles of at most L items when every row has fewer than s nonzeros)."""
    rp = np.ascontiguousarray(rp, dtype=np.int32)
    n = rp.size - 1
    total = n + int(rp[-1])
    T = (total + (L - slack) - 1) // (L - slack)
    ti = np.empty(T + 1, dtype=np.int32)
    tj = np.empty(T + 1, dtype=np.int32)
    lib().or_merge_tiles(n, _p(rp), L, slack, _p(ti), _p(tj))
    return ti, tj


def column_blocks(rp, col, val, B: int, width: int):
    """Column blocks (ML remedy on the merge path, Table II): block b holds,
    row by row in storage order, the nonzeros with column in
    [b width, (b + 1) width). Returns (rpb of shape (B, n + 1), each counting
    from 0, colb, valb with the blocks one after the other)."""
    rp = np.ascontiguousarray(rp, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    n = rp.size - 1
    rpb = np.zeros((B, n + 1), dtype=np.int32)
    colb = np.zeros(max(col.size, 1), dtype=np.int32)
    valb = np.zeros(max(col.size, 1), dtype=np.float64)
    lib().or_column_blocks(n, _p(rp), _p(col), _p(val), B, width, _p(rpb), _p(colb), _p(valb))
    return rpb, colb[:col.size], valb[:col.size]


def column_block_rows(rpb):
    """Row lists of column blocks 1 .. B-1 (blocks of split rows walk only
    the rows with nonzeros in them): per block the rows i with
    rpb[b, i+1] > rpb[b, i], ascending, and their row pointers from 0.
    Returns (rows, rowptr), the blocks one after the other."""
    rows, ptr = [], []
    for b in range(1, rpb.shape[0]):
        cnt = np.diff(rpb[b].astype(np.int64))
        r = np.nonzero(cnt)[0]
        rows.append(r.astype(np.int32))
        ptr.append(np.concatenate([[0], np.cumsum(cnt[r])]).astype(np.int32))
    cat = lambda a: np.concatenate(a) if a else np.zeros(0, dtype=np.int32)
    return cat(rows), cat(ptr)


def long_rows(rp, tau: int) -> np.ndarray:
    rp = np.ascontiguousarray(rp, dtype=np.int32)
    out = np.empty(max(rp.size - 1, 1), dtype=np.int32)
    k = lib().or_long_rows(rp.size - 1, _p(rp), tau, _p(out))
    return out[:k].copy()


def long_row_threshold(nnz_avg: float, factor: float = 32.0, floor: int = 4096) -> int:
    """tau = max(factor * nnz_avg, floor): a row is 'long' when it holds more
    nonzeros than this (the paper compares nnz_max against nnz_avg but states
    no number)."""
    return int(max(factor * nnz_avg, floor))


# ---------------------------------------------------------------------------
# Features (Sec. III-D, Table I)
# ---------------------------------------------------------------------------

FEATURE_NAMES = ("N", "nnz_min", "nnz_max", "nnz_avg", "nnz_sd", "bw_min", "bw_max",
                 "bw_avg", "bw_sd", "scatter_avg", "scatter_sd", "clustering_avg",
                 "misses_avg", "size", "mean_col_gap", "x_reuse")
FEATURE_INT_NAMES = ("sum_nnz", "sum_nnz2", "sum_bw", "sum_bw2", "sum_misses",
                     "sum_groups", "reuse_shared", "reuse_distinct")


def features(n_rows, n_cols, rp, col):
    """(16 FP64 features, 8 int64 sums) as defined in csr_oracle.c."""
    rp, col = _csr(rp, col)
    out = np.empty(16, dtype=np.float64)
    iout = np.empty(8, dtype=np.int64)
    lib().or_features(n_rows, n_cols, _p(rp), _p(col), _p(out), _p(iout))
    return out, iout


# ---------------------------------------------------------------------------
# Per-class bounds (Sec. III-B) and the profile-guided rule (Sec. III-C, Fig. 4)
# ---------------------------------------------------------------------------

MALL_BYTES = 256 * 1024 * 1024


def format_bytes(n_rows, n_cols, nnz, val_bytes=8, idx_bytes=4, extra=0):
    """S_format for CSR: values + indices + row pointers (+ any side table)."""
    return nnz * (val_bytes + idx_bytes) + 4 * (n_rows + 1) + extra


def p_mb(nnz, s_format, s_x, s_y, b_max):
    """P_MB = 2 NNZ / ((S_format + S_x + S_y) / B_max)  [flop/s]."""
    return 2.0 * nnz / ((s_format + s_x + s_y) / b_max)


def p_peak(nnz, s_values, s_x, s_y, b_max):
    """P_peak = 2 NNZ / ((S_values + S_x + S_y) / B_max): all indexing removed."""
    return 2.0 * nnz / ((s_values + s_x + s_y) / b_max)


def p_imb(nnz, unit_times):
    """P_IMB = 2 NNZ / t_median over the execution units that ran work; for an
    even count the median is the mean of the two middle values. Reading for a
    GPU: the paper's threads are the compute units, and a unit's time is the
    span from the start of its first workgroup to the end of its last one in
    the instrumented baseline run."""
    t = np.sort(np.asarray(unit_times, dtype=np.float64))
    if t.size == 0:
        return float("inf")
    m = t.size // 2
    med = t[m] if t.size % 2 else 0.5 * (t[m - 1] + t[m])
    return 2.0 * nnz / med


def b_for_footprint(bytes_total, b_hbm, b_cache, cache_bytes=MALL_BYTES):
    """B_max, raised to the cache bandwidth when the working set fits in the
    last-level cache (the footnote to the P_MB bound)."""
    return b_cache if bytes_total <= cache_bytes else b_hbm


def ml_partition_bounds(rp, rows_per_block: int, Q: int) -> np.ndarray:
    """Partition-aware ML detection, the extension the paper proposes with
    its Sec. IV-C results (look at the P_ML benchmark per partition instead
    of over the whole matrix). Reading: the partitions are Q contiguous runs
    of the baseline's row blocks (rows_per_block rows each) with about nnz/Q
    nonzeros each, as the static nnz-balanced partitioning of Sec. IV-A.
    bound[q] is the first block b (0 <= b <= nblk) whose first nonzero index
    rp[min(b * rows_per_block, N)] is at least floor(q * nnz / Q); bound[Q] is
    nblk. Linear scan over the blocks."""
    rp = np.asarray(rp, dtype=np.int64)
    n = rp.size - 1
    nnz = int(rp[-1])
    nblk = -(-n // rows_per_block)
    first = [int(rp[min(b * rows_per_block, n)]) for b in range(nblk + 1)]
    out = np.empty(Q + 1, dtype=np.int32)
    for q in range(Q):
        target = q * nnz // Q
        b = 0
        while b < nblk and first[b] < target:
            b += 1
        out[q] = b
    out[Q] = nblk
    return out


def ml_partition_ratios(t_base, t_probe, bounds) -> np.ndarray:
    """Per partition: the baseline's summed block times over the P_ML probe's
    summed block times (the P_ML / P_CSR ratio of Sec. III-B restricted to
    the partition); 0 for a partition without blocks or without time."""
    out = np.zeros(len(bounds) - 1)
    for q in range(len(bounds) - 1):
        sc = int(np.sum(np.asarray(t_base[bounds[q]:bounds[q + 1]], dtype=np.int64)))
        sm = int(np.sum(np.asarray(t_probe[bounds[q]:bounds[q + 1]], dtype=np.int64)))
        if sc > 0 and sm > 0:
            out[q] = sc / sm
    return out


CLS_MB, CLS_ML, CLS_IMB, CLS_CMP = 1, 2, 4, 8


def classify(p_csr, p_mb_, p_ml, p_imb_, p_cmp, p_peak_, t_ml=1.25, t_imb=1.24, t_mb=0.8):
    """Profile-guided classifier (Sec. III-C, Fig. 4) -> bit mask of classes.

    A matrix is in every class whose test on the bounds of Sec. III-B holds:
    imbalance and irregular x when removing them (P_IMB, P_ML) would beat
    the baseline by more than the thresholds; bandwidth when the baseline
    streams near P_MB and the no-index probe P_CMP lies between the two
    bandwidth bounds; computation when P_CMP lies outside them. The paper
    leaves its "approximately equal" undefined; read as P_CSR >= T_MB P_MB.
    """
    tests = {
        CLS_MB: p_csr >= t_mb * p_mb_ and p_mb_ < p_cmp < p_peak_,
        CLS_ML: p_ml / p_csr > t_ml,
        CLS_IMB: p_imb_ / p_csr > t_imb,
        CLS_CMP: p_cmp < p_mb_ or p_cmp > p_peak_,
    }
    return sum(cls for cls, holds in tests.items() if holds)


OPT_DELTA, OPT_PREFETCH, OPT_DECOMP, OPT_MERGE, OPT_UNROLL = 1, 2, 4, 8, 16
OPT_ORDER = (OPT_DELTA, OPT_PREFETCH, OPT_DECOMP, OPT_MERGE, OPT_UNROLL)


def remedies(classes: int, has_long_rows: bool, remedy_map: int = 0) -> int:
    """Class set -> optimization set, applied jointly.

    remedy_map 0 follows Sec. III-E, Table II:
      MB  -> delta-compressed column indices (+ wide loads)
      ML  -> prefetched x gathers
      IMB -> long-row decomposition when long rows exist, else the nnz-balanced
             merge-path split (the GPU counterpart of the runtime-chosen schedule)
      CMP -> unrolling with several rows per wavefront (+ wide loads)
    remedy_map 1 is the reading for a GPU on which prefetching and unrolling
    do not pay (Sec. III-C leaves the map to be fixed per platform):
      MB  -> delta-compressed column indices
      ML  -> the merge-path split with its codes (window-coded tiles gather
             x through one window brought into fast memory first)
      IMB -> decomposition when long rows exist, else merge path with codes
      CMP -> nothing
    """
    assert remedy_map in (0, 1)
    o = 0
    if classes & CLS_MB:
        o |= OPT_DELTA
    if remedy_map == 1:
        if classes & CLS_ML:
            o |= OPT_MERGE | OPT_DELTA
        if classes & CLS_IMB:
            o |= OPT_DECOMP if has_long_rows else (OPT_MERGE | OPT_DELTA)
        return o
    if classes & CLS_ML:
        o |= OPT_PREFETCH
    if classes & CLS_IMB:
        o |= OPT_DECOMP if has_long_rows else OPT_MERGE
    if classes & CLS_CMP:
        o |= OPT_UNROLL
    return o


def catalogue():
    """The K = 16 optimization sets the trivial optimizers of Sec. IV-D sweep:
    the baseline, the 5 singles and the 10 pairs (ids in this order)."""
    sets = [0] + list(OPT_ORDER)
    for a in range(5):
        for b in range(a + 1, 5):
            sets.append(OPT_ORDER[a] | OPT_ORDER[b])
    return sets


def n_iters_min(t_pre, t_base, t_opt):
    """Solver iterations needed to amortize the optimizer (Sec. IV-D, Eq. (2)):
    t_pre / (t_base - t_opt), infinite when the optimized SpMV is not faster."""
    if t_opt >= t_base:
        return float("inf")
    return t_pre / (t_base - t_opt)


def harmonic_mean(rates):
    """Run summary of Sec. IV-A: harmonic mean of the per-run rates."""
    r = np.asarray(rates, dtype=np.float64)
    return r.size / np.sum(1.0 / r)


# ---------------------------------------------------------------------------
# Learned selector: feature normalization and an FP64 MLP 16-64-64-K
# (replaces the decision tree of Sec. III-D; labels are timed-best variants)
# ---------------------------------------------------------------------------

def normalize(f, mu, sigma):
    """f' = (log2(1 + f) - mu) / sigma, per feature."""
    return (np.log2(1.0 + np.asarray(f, dtype=np.float64)) - mu) / sigma


def mlp_forward(params, X):
    """Hidden layers ReLU(W h + b), output logits W h + b. X: (B, in)."""
    h = np.asarray(X, dtype=np.float64)
    acts = [h]
    nl = len(params) // 2
    for l in range(nl):
        W, b = params[2 * l], params[2 * l + 1]
        z = h @ W.T + b
        h = np.maximum(z, 0.0) if l < nl - 1 else z
        acts.append(h)
    return h, acts


def softmax_xent(logits, labels):
    """Mean softmax cross-entropy and its gradient w.r.t. the logits."""
    z = logits - logits.max(axis=1, keepdims=True)
    e = np.exp(z)
    p = e / e.sum(axis=1, keepdims=True)
    B = logits.shape[0]
    loss = -np.mean(np.log(p[np.arange(B), labels]))
    g = p.copy()
    g[np.arange(B), labels] -= 1.0
    return loss, g / B


def mlp_loss_grad(params, X, labels):
    """Loss and gradients by the chain rule, layer by layer backwards."""
    logits, acts = mlp_forward(params, X)
    loss, g = softmax_xent(logits, labels)
    nl = len(params) // 2
    grads = [None] * len(params)
    for l in range(nl - 1, -1, -1):
        h_in = acts[l]
        W = params[2 * l]
        grads[2 * l] = g.T @ h_in
        grads[2 * l + 1] = g.sum(axis=0)
        if l > 0:
            g = (g @ W) * (acts[l] > 0.0)
    return loss, grads


def adam_step(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; t counts from 1."""
    out_p, out_m, out_v = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = b1 * mm + (1.0 - b1) * g
        vv = b2 * vv + (1.0 - b2) * g * g
        mh = mm / (1.0 - b1 ** t)
        vh = vv / (1.0 - b2 ** t)
        out_p.append(p - lr * mh / (np.sqrt(vh) + eps))
        out_m.append(mm)
        out_v.append(vv)
    return out_p, out_m, out_v


def regret(t_sel, t_best):
    """Per-matrix regret t_selected / t_best - 1."""
    return np.asarray(t_sel, dtype=np.float64) / np.asarray(t_best, dtype=np.float64) - 1.0

"""Seeded synthetic sparse matrices and vectors.

This module is shared by the CPU oracle tests and by the GPU path's tests and
benchmark. It only *produces inputs*: it holds none of the SpMV method's
arithmetic (no products, no partitioning, no encodings, no features).

Random numbers come from a counter-based generator: SplitMix64's output
finalizer (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) applied to a per-(seed, stream) base plus a counter,

    base(seed, stream) = mix64(seed * GAMMA + stream)
    h(seed, stream, i) = mix64(base + (i + 1) * GAMMA)      (mod 2**64)

so every draw is a pure function of (seed, stream, index) and any slice of a
matrix can be regenerated independently.

    u53      = h >> 11
    U(0,1]   = (u53 + 1) * 2**-53
    U[-1,1)  = u53 * 2**-52 - 1

The matrices stand in for the University of Florida (SuiteSparse) matrices the
paper measures on (Sec. IV-A, Sec. III-D "Training Data Selection"); none of
that collection is reproduced here. Each generator returns
``(n_rows, n_cols, row_ptr int32[N+1], col_idx int32[NNZ], val float64[NNZ])``
with columns sorted inside every row.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1

_U64 = np.uint64


def _mix64_int(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * M1) & MASK64
    z = ((z ^ (z >> 27)) * M2) & MASK64
    return z ^ (z >> 31)


def _mix64_arr(z: np.ndarray) -> np.ndarray:
    z = z ^ (z >> _U64(30))
    z = z * _U64(M1)
    z = z ^ (z >> _U64(27))
    z = z * _U64(M2)
    return z ^ (z >> _U64(31))


def stream_base(seed: int, stream: int) -> int:
    return _mix64_int((seed * GAMMA + stream) & MASK64)


def hash64(seed: int, stream: int, idx) -> np.ndarray:
    """h(seed, stream, i) for an integer array (or scalar) of indices i >= 0."""
    base = _U64(stream_base(seed, stream))
    i = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64_arr(base + (i + _U64(1)) * _U64(GAMMA))


def hash64_int(seed: int, stream: int, i: int) -> int:
    """Scalar twin of :func:`hash64` in plain Python integers."""
    return _mix64_int(stream_base(seed, stream) + ((i + 1) * GAMMA & MASK64))


def u01(seed: int, stream: int, idx) -> np.ndarray:
    """U(0,1] doubles."""
    u53 = (hash64(seed, stream, idx) >> _U64(11)).astype(np.float64)
    return (u53 + 1.0) * (2.0 ** -53)


def um11(seed: int, stream: int, idx) -> np.ndarray:
    """U[-1,1) doubles."""
    u53 = (hash64(seed, stream, idx) >> _U64(11)).astype(np.float64)
    return u53 * (2.0 ** -52) - 1.0


def uindex(seed: int, stream: int, idx, n: int) -> np.ndarray:
    """Integers uniform on [0, n)."""
    u53 = (hash64(seed, stream, idx) >> _U64(11)).astype(np.float64)
    v = np.floor(u53 * (2.0 ** -53) * n).astype(np.int64)
    return np.minimum(v, n - 1)


def vector(n: int, seed: int) -> np.ndarray:
    """x ~ U[-1,1) of length n."""
    return um11(seed, 0, np.arange(n, dtype=np.uint64))


def dyadic_vector(n: int, seed: int, kmax: int = 1024, shift: int = 10) -> np.ndarray:
    """x_i = k_i / 2**shift with integer |k_i| <= kmax (exactly representable)."""
    k = uindex(seed, 0, np.arange(n, dtype=np.uint64), 2 * kmax + 1) - kmax
    return k.astype(np.float64) / float(1 << shift)


# --------------------------------------------------------------------------
# CSR assembly helpers (pure bookkeeping: counting and ordering, no arithmetic
# of the method)
# --------------------------------------------------------------------------

def _from_sorted_keys(keys: np.ndarray, n_rows: int, n_cols: int):
    rows = (keys // n_cols).astype(np.int64)
    cols = (keys - rows * n_cols).astype(np.int32)
    counts = np.bincount(rows, minlength=n_rows).astype(np.int64)
    rp = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    return rp, cols


def _check_int32(rp: np.ndarray) -> np.ndarray:
    if rp[-1] >= 2 ** 31:
        raise ValueError("nnz does not fit int32 indices")
    return rp.astype(np.int32)


def from_coo(rows, cols, vals, n_rows: int, n_cols: int):
    """Sort (row, col) and build CSR; duplicates are kept (summed by SpMV)."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=n_rows)
    rp = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    return n_rows, n_cols, _check_int32(rp), cols.astype(np.int32), vals


def from_dense(a: np.ndarray):
    """CSR of the nonzero pattern of a small dense matrix (row-major order)."""
    a = np.asarray(a, dtype=np.float64)
    r, c = np.nonzero(a)
    return from_coo(r, c, a[r, c], a.shape[0], a.shape[1])


# --------------------------------------------------------------------------
# Configuration matrices
# --------------------------------------------------------------------------

def laplacian2d(nx: int = 100, ny: int | None = None):
    """5-point 2-D Laplacian on an nx-by-ny grid, row-major numbering.

    Diagonal 4, off-diagonals -1 (Dirichlet boundary: missing neighbours are
    dropped). 100x100 gives N = 10,000 and NNZ = 49,600.
    """
    ny = nx if ny is None else ny
    n = nx * ny
    idx = np.arange(n, dtype=np.int64)
    r, c = idx // nx, idx % nx
    offs = [(-1, 0), (0, -1), (0, 0), (0, 1), (1, 0)]  # ascending column order
    cols, vals, valid = [], [], []
    for dr, dc in offs:
        ok = (r + dr >= 0) & (r + dr < ny) & (c + dc >= 0) & (c + dc < nx)
        cols.append(idx + dr * nx + dc)
        vals.append(np.full(n, 4.0 if (dr, dc) == (0, 0) else -1.0))
        valid.append(ok)
    cols = np.stack(cols, 1)
    vals = np.stack(vals, 1)
    valid = np.stack(valid, 1)
    counts = valid.sum(1)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    return n, n, _check_int32(rp), cols[valid].astype(np.int32), vals[valid]


def stencil27(n: int = 128, seed_off: int = 201, seed_diag: int = 202):
    """27-point stencil on an n^3 grid (x fastest), columns ascending.

    Off-diagonal values U(0,1] drawn by CSR position (seed_off); the diagonal
    is (nnz_i - 1) + U(0,1] (seed_diag, by row), so each row is strictly
    diagonally dominant. 128^3 gives N = 2,097,152 and NNZ = 55,742,968.
    """
    N = n * n * n
    rp = np.zeros(N + 1, dtype=np.int64)
    idx = np.arange(N, dtype=np.int64)
    z, y, x = idx // (n * n), (idx // n) % n, idx % n
    del idx
    offs = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    vz = [(z + d >= 0) & (z + d < n) for d in (-1, 0, 1)]
    vy = [(y + d >= 0) & (y + d < n) for d in (-1, 0, 1)]
    vx = [(x + d >= 0) & (x + d < n) for d in (-1, 0, 1)]
    del z, y, x
    valid = np.empty((N, 27), dtype=bool)
    for k, (dz, dy, dx) in enumerate(offs):
        valid[:, k] = vz[dz + 1] & vy[dy + 1] & vx[dx + 1]
    del vz, vy, vx
    counts = valid.sum(1)
    np.cumsum(counts, out=rp[1:])
    nnz = int(rp[-1])
    offsets = np.array([(dz * n + dy) * n + dx for dz, dy, dx in offs], dtype=np.int64)
    # Column of each kept entry: row + offset of its stencil point.
    rows_of = np.repeat(np.arange(N, dtype=np.int64), counts)
    kk = np.nonzero(valid.ravel())[0] % 27
    col = (rows_of + offsets[kk]).astype(np.int32)
    is_diag = kk == 13
    del kk
    val = u01(seed_off, 0, np.arange(nnz, dtype=np.uint64))
    diag_rows = rows_of[is_diag]
    val[is_diag] = (counts[diag_rows] - 1).astype(np.float64) + u01(
        seed_diag, 0, diag_rows.astype(np.uint64))
    return N, N, _check_int32(rp), col, val


def rmat(scale: int = 22, edge_factor: int = 16, probs=(0.57, 0.19, 0.19, 0.05),
         seed_edges: int = 301, seed_vals: int = 302, chunk: int = 1 << 22):
    """R-MAT graph (Chakrabarti, Zhan & Faloutsos 2004) as a directed CSR matrix.

    edge_factor * 2^scale edges; for every edge and level l one 16-bit uniform
    u = (k + 0.5) / 65536 (four levels per 64-bit draw, stream l // 4) picks
    the quadrant a / b / c / d by cumulative probability. No vertex
    permutation and no noise; self-loops kept; duplicate (r, c) pairs merged
    into one entry whose value is U(0,1] drawn from (seed_vals, r * N + c).
    """
    N = 1 << scale
    m = edge_factor * N
    a, b, c, _ = probs
    t1 = a * 65536.0
    t2 = (a + b) * 65536.0
    t3 = (a + b + c) * 65536.0
    keys = []
    for e0 in range(0, m, chunk):
        e = np.arange(e0, min(m, e0 + chunk), dtype=np.uint64)
        r = np.zeros(e.shape, dtype=np.int64)
        cc = np.zeros(e.shape, dtype=np.int64)
        for s in range((scale + 3) // 4):
            h = hash64(seed_edges, s, e)
            for q in range(4):
                lvl = 4 * s + q
                if lvl >= scale:
                    break
                k = ((h >> _U64(16 * q)) & _U64(0xFFFF)).astype(np.float64) + 0.5
                row_bit = k >= t2                       # quadrants c, d
                col_bit = ((k >= t1) & (k < t2)) | (k >= t3)  # quadrants b, d
                bit = scale - 1 - lvl
                r |= row_bit.astype(np.int64) << bit
                cc |= col_bit.astype(np.int64) << bit
        keys.append(np.unique(r * N + cc))
    keys = np.unique(np.concatenate(keys))
    rp, col = _from_sorted_keys(keys, N, N)
    val = u01(seed_vals, 0, keys.astype(np.uint64))
    return N, N, _check_int32(rp), col, val


def uniform_random(n: int = 1 << 20, per_row: int = 16, seed_cols: int = 401,
                   seed_vals: int = 402, chunk: int = 1 << 18):
    """Exactly `per_row` distinct uniform columns per row (rejection sampling).

    Row i draws candidates c_k = uindex(seed_cols, stream=i, k) for
    k = 0, 1, 2, ... and keeps the first `per_row` distinct ones; columns are
    then sorted. Values U(0,1] by CSR position (seed_vals).
    """
    cols_all = []
    draws = per_row + 8
    for r0 in range(0, n, chunk):
        rows = np.arange(r0, min(n, r0 + chunk), dtype=np.int64)
        nr = rows.size
        # candidates[i, k]: per-row streams, so index = k, stream = row
        cand = np.empty((nr, draws), dtype=np.int64)
        for k in range(draws):
            cand[:, k] = _uindex_rows(seed_cols, rows, k, n)
        picked = _first_distinct(cand, per_row)
        while picked is None:  # astronomically rare: draw more
            draws += 8
            more = np.empty((nr, 8), dtype=np.int64)
            for k in range(8):
                more[:, k] = _uindex_rows(seed_cols, rows, draws - 8 + k, n)
            cand = np.concatenate([cand, more], 1)
            picked = _first_distinct(cand, per_row)
        cols_all.append(np.sort(picked, axis=1))
    col = np.concatenate(cols_all).reshape(-1).astype(np.int32)
    rp = (np.arange(n + 1, dtype=np.int64) * per_row)
    val = u01(seed_vals, 0, np.arange(col.size, dtype=np.uint64))
    return n, n, _check_int32(rp), col, val


def _uindex_rows(seed: int, rows: np.ndarray, k: int, n: int) -> np.ndarray:
    # one stream per row: base(seed, row) varies per element
    with np.errstate(over="ignore"):
        base = _mix64_arr(_U64((seed * GAMMA) & MASK64) + rows.astype(np.uint64))
    with np.errstate(over="ignore"):
        h = _mix64_arr(base + _U64((k + 1) * GAMMA & MASK64))
    u53 = (h >> _U64(11)).astype(np.float64)
    v = np.floor(u53 * (2.0 ** -53) * n).astype(np.int64)
    return np.minimum(v, n - 1)


def _first_distinct(cand: np.ndarray, k: int):
    nr, d = cand.shape
    order = np.lexsort((np.broadcast_to(np.arange(d), cand.shape).ravel(), cand.ravel(),
                        np.repeat(np.arange(nr), d)))
    flat = cand.ravel()[order]
    rowid = np.repeat(np.arange(nr), d)[order]
    dup_sorted = np.zeros(flat.size, dtype=bool)
    dup_sorted[1:] = (flat[1:] == flat[:-1]) & (rowid[1:] == rowid[:-1])
    dup = np.empty_like(dup_sorted)
    dup[order] = dup_sorted
    keep = ~dup.reshape(nr, d)
    rank = np.cumsum(keep, axis=1)
    if (rank[:, -1] < k).any():
        return None
    sel = keep & (rank <= k)
    return cand[sel].reshape(nr, k)


# --------------------------------------------------------------------------
# Families for the learned-selector suite and the batched launch
# --------------------------------------------------------------------------

def banded_random(n: int, bandwidth: int, per_row: int, seed: int, chunk: int = 1 << 18):
    """Row i draws `per_row` columns uniform in the window [i - bandwidth,
    i + bandwidth] clipped to [0, n) (draw t from stream 1 + t, index i) and
    keeps the distinct ones, sorted; a window no wider than per_row is taken
    whole. Values U(0,1] by CSR position."""
    rows_all, cols_all = [], []
    for r0 in range(0, n, chunk):
        rows = np.arange(r0, min(n, r0 + chunk), dtype=np.int64)
        lo = np.maximum(rows - bandwidth, 0)
        width = np.minimum(rows + bandwidth, n - 1) - lo + 1
        full = width <= per_row
        if full.any():
            fr, fw = rows[full], width[full]
            rr = np.repeat(fr, fw)
            offs = np.arange(rr.size) - np.repeat(np.cumsum(fw) - fw, fw)
            rows_all.append(rr)
            cols_all.append(np.repeat(lo[full], fw) + offs)
        part = ~full
        if part.any():
            pr, plo, pw = rows[part], lo[part], width[part]
            cand = np.empty((pr.size, per_row), dtype=np.int64)
            for t in range(per_row):
                u53 = (hash64(seed, 1 + t, pr.astype(np.uint64)) >> _U64(11)).astype(np.float64)
                cand[:, t] = plo + np.minimum(np.floor(u53 * 2.0 ** -53 * pw).astype(np.int64), pw - 1)
            cand.sort(axis=1)
            keep = np.ones(cand.shape, dtype=bool)
            keep[:, 1:] = cand[:, 1:] != cand[:, :-1]
            rows_all.append(np.broadcast_to(pr[:, None], cand.shape)[keep])
            cols_all.append(cand[keep])
    r = np.concatenate(rows_all)
    c = np.concatenate(cols_all)
    order = np.lexsort((c, r))
    r, c = r[order], c[order]
    vals = u01(seed, 0, np.arange(r.size, dtype=np.uint64))
    counts = np.bincount(r, minlength=n)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    return n, n, _check_int32(rp), c.astype(np.int32), vals


def localized_irregular(n: int, per_row: int, frac: float, seed: int):
    """Regular rows with an irregular stretch: every row holds exactly
    `per_row` columns; rows in [n/2, n/2 + frac*n) take distinct uniform
    random columns over [0, n) (rejection sampling as uniform_random, seed
    `seed`), the other rows the contiguous window starting at
    i - per_row/2, shifted to stay inside [0, n). Values U(0,1] by CSR
    position (seed + 1). The workload of the partition-aware ML test: the
    irregular gathers are confined to a few contiguous partitions."""
    r0 = n // 2
    r1 = min(n, r0 + int(round(frac * n)))
    rows = np.arange(n, dtype=np.int64)
    start = np.clip(rows - per_row // 2, 0, n - per_row)
    col = (start[:, None] + np.arange(per_row)[None, :]).astype(np.int64)
    if r1 > r0:
        irr = np.arange(r0, r1, dtype=np.int64)
        draws = per_row + 8
        cand = np.empty((irr.size, draws), dtype=np.int64)
        for k in range(draws):
            cand[:, k] = _uindex_rows(seed, irr, k, n)
        picked = _first_distinct(cand, per_row)
        while picked is None:  # astronomically rare: draw more
            draws += 8
            more = np.empty((irr.size, 8), dtype=np.int64)
            for k in range(8):
                more[:, k] = _uindex_rows(seed, irr, draws - 8 + k, n)
            cand = np.concatenate([cand, more], 1)
            picked = _first_distinct(cand, per_row)
        col[r0:r1] = np.sort(picked, axis=1)
    rp = np.arange(n + 1, dtype=np.int64) * per_row
    val = u01(seed + 1, 0, np.arange(n * per_row, dtype=np.uint64))
    return n, n, _check_int32(rp), col.reshape(-1).astype(np.int32), val


def block_diagonal(n: int, block: int, seed: int):
    """Dense block x block blocks along the diagonal (last block clipped)."""
    rows = np.arange(n, dtype=np.int64)
    b0 = (rows // block) * block
    b1 = np.minimum(b0 + block, n)
    counts = b1 - b0
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    nnz = int(rp[-1])
    offs = np.arange(nnz, dtype=np.int64) - np.repeat(rp[:-1], counts)
    col = (np.repeat(b0, counts) + offs).astype(np.int32)
    val = u01(seed, 0, np.arange(nnz, dtype=np.uint64))
    return n, n, _check_int32(rp), col, val


def power_law(n: int, alpha: float, seed: int, max_nnz: int | None = None):
    """Row lengths from a discrete Pareto law (minimum 1, capped at n or
    max_nnz), columns uniform without replacement per row (rejection by
    sorting and de-duplicating, then topping up), values U(0,1]."""
    cap = n if max_nnz is None else min(n, max_nnz)
    u = u01(seed, 1, np.arange(n, dtype=np.uint64))
    lens = np.minimum(np.floor(u ** (-1.0 / alpha)).astype(np.int64), cap)
    lens = np.maximum(lens, 1)
    rows = np.repeat(np.arange(n, dtype=np.int64), lens)
    pos = np.arange(rows.size, dtype=np.uint64)
    cols = uindex(seed, 2, pos, n)
    keys = np.unique(rows * n + cols)
    rp, col = _from_sorted_keys(keys, n, n)
    val = u01(seed, 0, np.arange(col.size, dtype=np.uint64))
    return n, n, _check_int32(rp), col, val


def suite_matrix(index: int, base_seed: int = 501, n_min: float = 1e4, n_max: float = 4e6,
                 nnz_cap: int = 1 << 25):
    """Matrix `index` of the mixed learned-selector suite.

    Families (index % 5): 2-D/3-D stencils, banded random (bandwidth
    log-uniform 8..4096, 4..64 nnz/row), R-MAT (edge factor 4..32, jittered
    a,b,c,d), block-diagonal (blocks 4/8/16/32), power-law row lengths
    (Pareto alpha in [1.5, 3]). N log-uniform in [n_min, n_max]; sizes are
    reduced where needed so that NNZ stays within nnz_cap.
    Returns (name, matrix tuple).
    """
    seed = base_seed + index
    fam = index % 5
    p = u01(seed, 7, np.arange(8, dtype=np.uint64))
    n = int(math.exp(math.log(n_min) + (math.log(n_max) - math.log(n_min)) * p[0]))
    if fam == 0:
        kind = int(p[1] * 4) % 4
        if kind == 0:
            s = max(8, int(round(math.sqrt(min(n, nnz_cap // 5)))))
            return f"lap2d_{s}", laplacian2d(s)
        if kind == 1:
            s = max(8, int(round(math.sqrt(min(n, nnz_cap // 9)))))
            return f"nine2d_{s}", _nine_point(s, seed)
        if kind == 2:
            s = max(4, int(round(min(n, nnz_cap // 7) ** (1 / 3))))
            return f"seven3d_{s}", _seven_point(s, seed)
        s = max(4, int(round(min(n, nnz_cap // 27) ** (1 / 3))))
        return f"st27_{s}", stencil27(s, seed, seed + 100000)
    if fam == 1:
        bw = int(math.exp(math.log(8) + (math.log(4096) - math.log(8)) * p[1]))
        k = int(math.exp(math.log(4) + (math.log(64) - math.log(4)) * p[2]))
        k = max(1, min(k, 2 * bw + 1, nnz_cap // n))
        return f"band_{n}_{bw}_{k}", banded_random(n, bw, k, seed)
    if fam == 2:
        scale = max(10, int(round(math.log2(n))))
        ef = 4 + int(p[1] * 29) % 29
        while ef * (1 << scale) > nnz_cap:
            scale -= 1
        j = (p[2:6] - 0.5) * 0.1
        pr = np.array([0.57, 0.19, 0.19, 0.05]) + j
        pr = np.maximum(pr, 0.01)
        pr = pr / pr.sum()
        return f"rmat_{scale}_{ef}", rmat(scale, ef, tuple(pr), seed, seed + 100000)
    if fam == 3:
        blk = (4, 8, 16, 32)[int(p[1] * 4) % 4]
        n = min(n, nnz_cap // blk)
        return f"bdiag_{n}_{blk}", block_diagonal(n, blk, seed)
    alpha = 1.5 + 1.5 * p[1]
    return f"plaw_{n}_{alpha:.2f}", power_law(n, alpha, seed, max_nnz=max(64, nnz_cap // max(n, 1)))


def _nine_point(s: int, seed: int):
    n = s * s
    idx = np.arange(n, dtype=np.int64)
    r, c = idx // s, idx % s
    cols, valid = [], []
    for dr in (-1, 0, 1):
        for dc in (-1, 0, 1):
            valid.append((r + dr >= 0) & (r + dr < s) & (c + dc >= 0) & (c + dc < s))
            cols.append(idx + dr * s + dc)
    cols = np.stack(cols, 1)
    valid = np.stack(valid, 1)
    counts = valid.sum(1)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    col = cols[valid].astype(np.int32)
    val = u01(seed, 0, np.arange(col.size, dtype=np.uint64))
    return n, n, _check_int32(rp), col, val


def _seven_point(s: int, seed: int):
    n = s * s * s
    idx = np.arange(n, dtype=np.int64)
    z, y, x = idx // (s * s), (idx // s) % s, idx % s
    offs = [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 0), (0, 0, 1), (0, 1, 0), (1, 0, 0)]
    cols, valid = [], []
    for dz, dy, dx in offs:
        valid.append((z + dz >= 0) & (z + dz < s) & (y + dy >= 0) & (y + dy < s)
                     & (x + dx >= 0) & (x + dx < s))
        cols.append(idx + (dz * s + dy) * s + dx)
    cols = np.stack(cols, 1)
    valid = np.stack(valid, 1)
    counts = valid.sum(1)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    col = cols[valid].astype(np.int32)
    val = u01(seed, 0, np.arange(col.size, dtype=np.uint64))
    return n, n, _check_int32(rp), col, val


def laplacian3d(s: int = 128):
    """7-point 3-D Laplacian on an s^3 grid (x fastest), columns ascending.

    Diagonal 6, off-diagonals -1, Dirichlet boundary (missing neighbours
    dropped): symmetric positive definite. 128^3 gives N = 2,097,152 and
    NNZ = 14,581,760.
    """
    n, _, rp, col, _ = _seven_point(s, 0)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp.astype(np.int64)))
    val = np.where(col == rows, 6.0, -1.0)
    return n, n, rp, col, val


def spd_stencil27(s: int = 128, seed: int = 211):
    """Symmetric positive definite matrix on the 27-point pattern of an s^3
    grid: a_ij = a_ji = -U(0,1] drawn from the unordered pair (i, j), and
    a_ii = 1 + sum_j |a_ij| (strictly diagonally dominant with a positive
    diagonal, hence SPD). The pattern and sizes are those of stencil27(s).
    """
    n, _, rp, col, _ = stencil27(s)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp.astype(np.int64)))
    c = col.astype(np.int64)
    lo, hi = np.minimum(rows, c), np.maximum(rows, c)
    val = -u01(seed, 0, (lo * n + hi).astype(np.uint64))
    diag = c == rows
    val[diag] = 0.0
    rowsum = np.add.reduceat(np.abs(val), rp[:-1].astype(np.int64))
    val[diag] = 1.0 + rowsum[rows[diag]]
    return n, n, rp, col, val


def batch_matrix(index: int, base_seed: int = 601):
    """Matrix `index` of the batched-launch set: suite families, N log-uniform
    in [1024, 65536]."""
    return suite_matrix(index, base_seed=base_seed, n_min=1024, n_max=65536)


def tiny_random(m: int, n: int, density: float, seed: int, dyadic: bool = False,
                empty_rows: bool = True):
    """Small random CSR for brute-force checks. Values U[-1,1) or, if dyadic,
    small integers in [-8, 8] (exact in every storage precision)."""
    cnt = m * n
    u = u01(seed, 0, np.arange(cnt, dtype=np.uint64)).reshape(m, n)
    mask = u <= density
    if not empty_rows and m > 0 and n > 0:
        empty = ~mask.any(1)
        mask[empty, uindex(seed, 3, np.nonzero(empty)[0].astype(np.uint64), n)] = True
    if dyadic:
        v = (uindex(seed, 1, np.arange(cnt, dtype=np.uint64), 17) - 8).astype(np.float64)
        v[v == 0] = 1.0
    else:
        v = um11(seed, 1, np.arange(cnt, dtype=np.uint64))
    v = v.reshape(m, n)
    r, c = np.nonzero(mask)
    return from_coo(r, c, v[r, c], m, n)


def mlp_init_weights(sizes, seed: int = 701):
    """He-uniform initial weights for an MLP with layer widths `sizes`:
    W_l ~ U[-sqrt(6/fan_in), sqrt(6/fan_in)) of shape (fan_out, fan_in), drawn
    with stream = layer and index = flat position; biases zero. These are the
    random draws of training, passed as inputs to both the oracle and the GPU
    trainer. Returns [W1, b1, W2, b2, ...] as float64 arrays."""
    params = []
    for l in range(len(sizes) - 1):
        fi, fo = sizes[l], sizes[l + 1]
        lim = math.sqrt(6.0 / fi)
        w = um11(seed, l, np.arange(fo * fi, dtype=np.uint64)).reshape(fo, fi) * lim
        params += [w, np.zeros(fo)]
    return params


def permutation(n: int, seed: int, stream: int = 0) -> np.ndarray:
    """Seeded Fisher-Yates shuffle of range(n): for k = n-1 .. 1 swap k with
    uindex(seed, stream, k, k + 1)."""
    p = np.arange(n, dtype=np.int64)
    if n < 2:
        return p
    js = uindex_vec(seed, stream, np.arange(n, dtype=np.uint64), np.arange(n, dtype=np.int64) + 1)
    for k in range(n - 1, 0, -1):
        j = int(js[k])
        p[k], p[j] = p[j], p[k]
    return p


def uindex_vec(seed: int, stream: int, idx, n) -> np.ndarray:
    """Integers uniform on [0, n_i) with a per-element bound n_i."""
    u53 = (hash64(seed, stream, idx) >> _U64(11)).astype(np.float64)
    n = np.asarray(n, dtype=np.int64)
    v = np.floor(u53 * (2.0 ** -53) * n).astype(np.int64)
    return np.minimum(v, n - 1)

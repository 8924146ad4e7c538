"""Pins of the oracle's storage transforms: FP32/BF16 rounding, delta-coded
column indices (Sec. III-E, Table II: MB remedy), merge-path tiles and the
long-row list (Sec. III-E: IMB remedies)."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- precision

def test_f32_matches_numpy_cast():
    v = np.concatenate([synth.vector(100000, 1) * np.exp2(
        synth.uindex(2, 0, np.arange(100000, dtype=np.uint64), 300) - 150),
        [0.0, -0.0, np.inf, -np.inf, 1e-46, 3.4028235677973366e38, 1e39]])
    with np.errstate(over="ignore"):
        ref = v.astype(np.float32)
    assert np.array_equal(oracle.to_f32(v).view(np.uint32), ref.view(np.uint32))


def test_bf16_matches_torch_on_f32_representable_values():
    # For values already exact in FP32 a single rounding to BF16 is what
    # torch's float32 -> bfloat16 conversion (round to nearest even) does.
    f = (synth.vector(200000, 3) * np.exp2(
        synth.uindex(4, 0, np.arange(200000, dtype=np.uint64), 250) - 125)).astype(np.float32)
    ref = torch.from_numpy(f).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    got = oracle.to_bf16_bits(f.astype(np.float64))
    assert np.array_equal(got, ref)


def _bf16_finite_table():
    bits = np.arange(1 << 16, dtype=np.uint32)
    with np.errstate(invalid="ignore"):
        w = (bits << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    ok = np.isfinite(w) & (w >= 0) & ~((bits == 0x8000))
    b = bits[ok & (bits < 0x8000)]
    vals = w[ok & (bits < 0x8000)]
    order = np.argsort(vals)
    return vals[order], b[order].astype(np.uint16)


def test_bf16_brute_force_nearest_even():
    # Brute force over the table of all finite non-negative BF16 values: the
    # nearest one, ties to the even bit pattern, overflow past the halfway
    # point above the largest finite value to infinity.
    vals, bits = _bf16_finite_table()
    n = 20000
    mag = np.exp2(synth.uindex(6, 0, np.arange(n, dtype=np.uint64), 280) - 140)
    v = np.abs(synth.vector(n, 5)) * mag
    # plus exact halfway points and points next to them
    k = synth.uindex(7, 0, np.arange(2000, dtype=np.uint64), vals.size - 1)
    mids = 0.5 * (vals[k] + vals[k + 1])
    v = np.concatenate([v, mids, np.nextafter(mids, 0), np.nextafter(mids, np.inf)])
    got = oracle.to_bf16_bits(v)
    hi = np.searchsorted(vals, v, side="left")
    expect = np.empty(v.size, dtype=np.uint16)
    top = vals[-1]
    half_over = top + 0.5 * (top - vals[-2])
    for q in range(v.size):
        x = v[q]
        if x >= half_over:
            expect[q] = 0x7F80
            continue
        h = min(hi[q], vals.size - 1)
        lo = max(h - 1, 0)
        cands = [(abs(vals[c] - x), c) for c in {lo, h}]
        cands.sort(key=lambda t: t[0])
        if len(cands) == 2 and cands[0][0] == cands[1][0]:
            c = cands[0][1] if bits[cands[0][1]] % 2 == 0 else cands[1][1]
        else:
            c = cands[0][1]
        expect[q] = bits[c]
    assert np.array_equal(got, expect)
    # negative values mirror the sign bit
    assert np.array_equal(oracle.to_bf16_bits(-v), expect | 0x8000)


def test_bf16_edge_table():
    cases = {
        1.0: 0x3F80,
        1.0 + 2.0 ** -8: 0x3F80,                    # halfway, even stays
        1.0 + 3 * 2.0 ** -8: 0x3F82,                # halfway, odd rounds up
        1.0 + 2.0 ** -8 + 2.0 ** -40: 0x3F81,       # single rounding (FP32 first would give 0x3F80)
        (2 - 2.0 ** -7) * 2.0 ** 127: 0x7F7F,       # largest finite
        (2 - 2.0 ** -8) * 2.0 ** 127: 0x7F80,       # halfway above it: to even = inf
        np.nextafter((2 - 2.0 ** -8) * 2.0 ** 127, 0): 0x7F7F,
        2.0 ** -133: 0x0001,                        # smallest subnormal
        2.0 ** -134: 0x0000,                        # halfway to zero: even
        1.5 * 2.0 ** -134: 0x0001,
        2.0 ** -126: 0x0080,                        # smallest normal
        -0.0: 0x8000,
        np.inf: 0x7F80,
        -np.inf: 0xFF80,
        float("nan"): 0x7FC0,
    }
    v = np.array(list(cases.keys()), dtype=np.float64)
    got = oracle.to_bf16_bits(v)
    assert [int(g) for g in got] == list(cases.values())
    back = oracle.bf16_bits_to_f64(np.array([0x3F81, 0x0001, 0xC000], dtype=np.uint16))
    assert list(back) == [1.0 + 2.0 ** -7, 2.0 ** -133, -2.0]


def test_reduced_precision_bound_holds_for_sequential_fp32():
    # numpy float32 accumulation in storage order is one admissible FP32
    # summation; it must sit inside the a-priori bound.
    n, _, rp, col, val = synth.stencil27(12)
    x = synth.vector(n, 9)
    for storage in ("f32", "bf16"):
        vq = oracle.quantize(val, storage).astype(np.float32)
        xq = x.astype(np.float32)
        y = np.zeros(n, dtype=np.float32)
        prods = vq * xq[col]
        for i in range(n):
            s = np.float32(0)
            for p in prods[rp[i]:rp[i + 1]]:
                s = np.float32(s + p)
            y[i] = s
        yq, bound = oracle.reduced_precision_bound(rp, col, val, x, storage)
        assert np.all(np.abs(y.astype(np.float64) - yq) <= bound)


# ---------------------------------------------------------------- delta codes

def test_delta_round_trip_laplacian_w8():
    n, _, rp, col, _ = synth.laplacian2d(100)
    assert oracle.delta_width(rp, col) == 8
    codes = oracle.delta_encode(rp, col, 8)
    assert codes.dtype == np.uint8
    assert np.array_equal(oracle.delta_decode(rp, codes, 8), col)
    # closed form: first offsets in [-100, 0], gaps 1, 99 or 100
    first = codes[rp[:-1]].view(np.int8)
    assert first.min() == -100 and first.max() == 0
    rest = np.delete(codes, rp[:-1])
    assert set(np.unique(rest).tolist()) == {1, 99, 100}


def test_delta_stencil27_w16_closed_form():
    # 27-point stencil on n^3: the most negative first offset is -(n^2+n+1)
    # and the largest gap is n^2 - n - 1 (a row on the y=0 or y=n-1 face with
    # x at a face, jumping from plane z-1 to plane z): 16,513 and 16,255 for
    # n = 128, so 16-bit codes fit and 8-bit ones do not.
    gold = json.load(open(os.path.join(GOLDEN, "stencil27_delta.json")))
    n = gold["n"]
    N, _, rp, col, _ = synth.stencil27(n)
    assert not oracle.delta_eligible(rp, col, 8)
    codes = oracle.delta_encode(rp, col, 16)
    first = codes[rp[:-1]].view(np.int16)
    rest = np.delete(codes, rp[:-1])
    assert int(first.min()) == gold["min_first_offset"]
    assert int(rest.max()) == gold["max_gap"]
    assert np.array_equal(oracle.delta_decode(rp, codes, 16), col)


@pytest.mark.parametrize("w", [8, 16])
def test_delta_boundaries(w):
    lo, umax = -(1 << (w - 1)), (1 << w) - 1
    ncol = 1 << 20
    # row 0 at the signed limit, then a gap at the unsigned limit
    row = 1 << (w - 1)
    rp = np.array([0] * (row + 1) + [2], dtype=np.int32)
    ok = np.array([row + lo, row + lo + umax], dtype=np.int32)
    assert oracle.delta_eligible(rp, ok, w)
    codes = oracle.delta_encode(rp, ok, w)
    assert np.array_equal(oracle.delta_decode(rp, codes, w), ok)
    assert not oracle.delta_eligible(rp, np.array([row + lo - 1, row + lo + umax - 1], dtype=np.int32), w)
    assert not oracle.delta_eligible(rp, np.array([row + lo, row + lo + umax + 1], dtype=np.int32), w)
    # positive signed limit
    assert oracle.delta_eligible(rp, np.array([row + (-lo - 1), row + (-lo - 1) + 1], dtype=np.int32), w)
    assert not oracle.delta_eligible(rp, np.array([row - lo, row - lo + 1], dtype=np.int32), w)
    # duplicates and unsorted rows are not encodable
    assert not oracle.delta_eligible(rp, np.array([row, row], dtype=np.int32), w)
    assert not oracle.delta_eligible(rp, np.array([row + 1, row], dtype=np.int32), w)
    assert ncol > 0


def test_irregular_matrices_are_not_delta_eligible():
    _, _, rp, col, _ = synth.uniform_random(1 << 17, 16)
    assert oracle.delta_width(rp, col) == 32


# ---------------------------------------------------------------- merge path

def _merge_path_by_steps(rp):
    """Walk the merge of row ends and nonzeros one item at a time: a nonzero
    j is consumed while j < rp[i+1], otherwise the row end i."""
    n = len(rp) - 1
    nnz = int(rp[-1])
    i = j = 0
    path = [(0, 0)]
    while i < n or j < nnz:
        if i < n and j >= rp[i + 1]:
            i += 1
        elif j < nnz:
            j += 1
        else:
            i += 1
        path.append((i, j))
    return path


@pytest.mark.parametrize("case", range(8))
def test_merge_tiles_match_step_simulation(case):
    if case == 0:
        rp = np.array([0], dtype=np.int32)                       # empty matrix
    elif case == 1:
        rp = np.array([0, 0, 0, 0], dtype=np.int32)              # only empty rows
    elif case == 2:
        rp = np.array([0, 50], dtype=np.int32)                   # one long row
    elif case == 3:
        rp = np.array([0, 3, 3, 3, 10, 11, 11], dtype=np.int32)  # mixed
    else:
        m, n, rp, _, _ = synth.tiny_random(30 + 7 * case, 40, 0.05 * case, case)
    path = _merge_path_by_steps(rp)
    assert path[-1] == (len(rp) - 1, int(rp[-1]))
    ti, tj = oracle.merge_tiles(rp, 1)
    assert list(zip(ti.tolist(), tj.tolist())) == path
    for L in (2, 3, 7, 64):
        ti, tj = oracle.merge_tiles(rp, L)
        total = len(path) - 1
        want = [path[min(t * L, total)] for t in range(len(ti))]
        assert list(zip(ti.tolist(), tj.tolist())) == want
        assert len(ti) == (total + L - 1) // L + 1


def _first_row_start_from(path, rp, p):
    """Index of the first point at or after step p of the path that is a row
    start (j == rp[i], row i not begun) or the end of the path."""
    n = len(rp) - 1
    for q in range(p, len(path)):
        i, j = path[q]
        if i == n or j == rp[i]:
            return q
    return len(path) - 1


@pytest.mark.parametrize("case", range(6))
def test_row_aligned_tiles_by_path_walk(case):
    if case == 0:
        rp = np.array([0, 3, 3, 3, 10, 11, 11, 11, 14], dtype=np.int32)  # empty rows
    elif case == 1:
        rp = np.arange(0, 41, 4, dtype=np.int32)                          # equal rows
    else:
        _, _, rp, _, _ = synth.tiny_random(40 + 9 * case, 50, 0.04 * case, 70 + case)
    n, nnz = len(rp) - 1, int(rp[-1])
    s = int(np.diff(rp).max()) + 1            # every row has fewer than s nonzeros
    path = _merge_path_by_steps(rp)
    total = len(path) - 1
    for L in (s + 1, s + 5, 64):
        ti, tj = oracle.merge_tiles(rp, L, s)
        pts = list(zip(ti.tolist(), tj.tolist()))
        assert len(pts) == (total + (L - s) - 1) // (L - s) + 1
        for t, pt in enumerate(pts):          # the cut at t(L-s), moved to a row start
            assert pt == path[_first_row_start_from(path, rp, min(t * (L - s), total))]
        assert pts[0] == (0, 0) and pts[-1] == (n, nnz)
        for i, j in pts:                      # no tile cuts a row
            assert i == n or j == rp[i]
        sizes = np.diff(ti.astype(np.int64) + tj)
        assert np.all(sizes >= 0) and np.all(sizes <= L)
    # slack 0 is the plain partition
    for L in (3, 7):
        a, b = oracle.merge_tiles(rp, L, 0), oracle.merge_tiles(rp, L)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_merge_tiles_invariants_on_rmat():
    n, _, rp, _, _ = synth.rmat(14, 16)
    L = 256
    ti, tj = oracle.merge_tiles(rp, L)
    assert ti[0] == 0 and tj[0] == 0
    assert ti[-1] == n and tj[-1] == rp[-1]
    assert np.all(np.diff(ti) >= 0) and np.all(np.diff(tj) >= 0)
    steps = np.diff(ti.astype(np.int64) + tj)
    assert np.all(steps[:-1] == L) and 0 < steps[-1] <= L
    # sampled diagonals against the step rule
    rp64 = rp.astype(np.int64)
    for t in range(0, len(ti), 97):
        i, j = int(ti[t]), int(tj[t])
        # all row ends before i are consumed: rp[i] <= j; row end i is not: j <= rp[i+1] (when i<n)
        assert i == n or j <= rp64[i + 1]
        assert i == 0 or rp64[i] <= j


# ---------------------------------------------------------------- long rows

def test_long_rows_hand_built():
    lens = [1, 5000, 3, 0, 4097, 4096, 9999]
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    assert oracle.long_rows(rp, 4096).tolist() == [1, 4, 6]
    assert oracle.long_rows(rp, 100000).tolist() == []
    assert oracle.long_row_threshold(4.0) == 4096
    assert oracle.long_row_threshold(1000.0) == 32000


# ------------------------------------------------------- tile-base column codes

def _tile_of_each_nonzero(tj, nnz):
    return np.repeat(np.arange(len(tj) - 1), np.diff(tj.astype(np.int64)))[:nnz]


@pytest.mark.parametrize("name,L,w", [("lap", 256, 16), ("lap", 512, 16), ("st27", 512, 16),
                                       ("rand", 64, 8)])
def test_merge_codes_round_trip_and_minimum(name, L, w):
    if name == "lap":
        n, _, rp, col, _ = synth.laplacian2d(100)
    elif name == "st27":
        n, _, rp, col, _ = synth.stencil27(12)
    else:
        n, _, rp, col, _ = synth.tiny_random(200, 40, 0.05, 3)
    ti, tj = oracle.merge_tiles(rp, L)
    got = oracle.merge_codes(tj, col, w)
    assert got is not None
    base, codes = got
    t_of = _tile_of_each_nonzero(tj, len(col))
    # decode(encode(col)) == col
    assert np.array_equal(base[t_of].astype(np.int64) + codes.astype(np.int64), col)
    # base_t is the smallest column of a non-empty tile: one code is 0
    for t in range(len(tj) - 1):
        if tj[t + 1] > tj[t]:
            assert codes[tj[t]:tj[t + 1]].min() == 0


def test_merge_codes_width_boundaries():
    # one row, tile = whole matrix: columns {0, 2^w - 1} fit, {0, 2^w} do not
    for w in (8, 16):
        for top, ok in (((1 << w) - 1, True), (1 << w, False)):
            rp = np.array([0, 2], dtype=np.int32)
            col = np.array([0, top], dtype=np.int32)
            ti, tj = oracle.merge_tiles(rp, 8)
            assert (oracle.merge_codes(tj, col, w) is not None) == ok


def test_merge_codes_laplacian_and_stencil_ranges():
    # 5-point Laplacian on n x n: a tile holding rows [i0, i1) touches
    # columns within [i0 - n, i1 - 1 + n], a range of at most rows - 1 + 2n
    n = 100
    _, _, rp, col, _ = synth.laplacian2d(n)
    ti, tj = oracle.merge_tiles(rp, 256)
    base, codes = oracle.merge_codes(tj, col, 16)
    t_of = _tile_of_each_nonzero(tj, len(col))
    rng = np.zeros(len(tj) - 1, dtype=np.int64)
    np.maximum.at(rng, t_of, codes.astype(np.int64))
    rows_touched = np.diff(ti.astype(np.int64)) + 1
    assert np.all(rng <= rows_touched - 1 + 2 * n)
    # 27-point on m^3: offsets reach +-(m^2 + m + 1); 16-bit fits, 8-bit does not
    m = 20
    _, _, rp, col, _ = synth.stencil27(m)
    ti, tj = oracle.merge_tiles(rp, 512)
    assert oracle.merge_codes(tj, col, 16) is not None
    assert oracle.merge_codes(tj, col, 8) is None


# ------------------------------------------------- window codes (row-aligned tiles)

def _aligned_tiles(rp, L):
    """Row-aligned merge tiles: slack = longest row + 1 (rows under 64 nonzeros)."""
    s = int(np.diff(rp.astype(np.int64)).max()) + 1
    assert s <= 64 and s < L
    return oracle.merge_tiles(rp, L, s)


@pytest.mark.parametrize("name,L", [("lap", 256), ("lap", 512), ("st27", 512), ("rand", 128)])
def test_window_codes_decode_and_window_order(name, L):
    if name == "lap":
        n, _, rp, col, _ = synth.laplacian2d(60)
    elif name == "st27":
        n, _, rp, col, _ = synth.stencil27(12)
    else:
        n, _, rp, col, _ = synth.tiny_random(300, 2000, 0.01, 5)
    ti, tj = _aligned_tiles(rp, L)
    got = oracle.window_codes(tj, col)
    assert got is not None
    base, wlen, dct, codes = got
    t_of = _tile_of_each_nonzero(tj, len(col))
    # decode: base_t + dict[t, code_j] == col_j, and every code lies in the window
    assert np.all(codes < wlen[t_of])
    assert np.array_equal(base[t_of].astype(np.int64) + dct[t_of, codes].astype(np.int64), col)
    for t in range(len(tj) - 1):
        w = dct[t, :wlen[t]].astype(np.int64)
        cols = col[tj[t]:tj[t + 1]]
        # the window is exactly the tile's distinct columns, ascending (brute force)
        assert list(w + base[t]) == sorted(set(int(c) for c in cols))
        assert np.all(dct[t, wlen[t]:] == 0)


def test_window_codes_laplacian_closed_form():
    # 5-point Laplacian on n x n, row r = (y, x): columns r - n, r - 1, r, r + 1,
    # r + n where they exist. A row-aligned tile holding rows [a, b) of one grid
    # interior (1 <= x, y and x, y <= n - 2 for every row, b - a + 2 < n) has the
    # three disjoint bands [a-n, b-1-n], [a-1, b], [a+n, b-1+n]: 3 (b - a) + 2
    # distinct columns, the smallest a - n.
    n = 100
    _, _, rp, col, _ = synth.laplacian2d(n)
    ti, tj = _aligned_tiles(rp, 256)
    base, wlen, _, _ = oracle.window_codes(tj, col)
    checked = 0
    for t in range(len(tj) - 1):
        a, b = int(ti[t]), int(ti[t + 1])
        rows = np.arange(a, b)
        if b <= a or b - a + 2 >= n:
            continue
        x, y = rows % n, rows // n
        if x.min() < 1 or x.max() > n - 2 or y.min() < 1 or y.max() > n - 2:
            continue
        assert wlen[t] == 3 * (b - a) + 2
        assert base[t] == a - n
        checked += 1
    assert checked > 10


def test_window_codes_boundaries():
    # one row per case; tile = whole matrix (L well above the row)
    def one_row(cols):
        rp = np.array([0, len(cols)], dtype=np.int32)
        c = np.array(cols, dtype=np.int32)
        ti, tj = oracle.merge_tiles(rp, 1024, len(cols) + 1)
        return oracle.window_codes(tj, c)
    # width: 256 distinct columns fit, 257 do not (maxw = 256)
    assert one_row(list(range(0, 512, 2))) is not None          # 256 distinct
    assert one_row(list(range(0, 514, 2))) is None              # 257 distinct
    # range: max - min = 2^16 - 1 fits, 2^16 does not
    assert one_row([5, 5 + 65535]) is not None
    assert one_row([5, 5 + 65536]) is None
    # repeated columns share one window entry and one code
    base, wlen, dct, codes = one_row([7, 9, 9, 7, 12])
    assert base[0] == 7 and wlen[0] == 3
    assert list(dct[0, :3]) == [0, 2, 5] and list(codes) == [0, 1, 1, 0, 2]


# ------------------------------------------------- run windows (row-aligned tiles)

def _expand_runs(rec):
    """The window a run record describes: base + start_r + k for k < len_r."""
    base, m, nr = int(rec[0]), int(rec[1]) & 0xFFFF, int(rec[1]) >> 16
    cols = []
    for r in range(nr):
        start, ln = int(rec[2 + r]) & 0xFFFF, (int(rec[2 + r]) >> 16) & 0xFFFF
        cols += [base + start + k for k in range(ln)]
    assert len(cols) == m
    assert all(int(v) == 0 for v in rec[2 + nr:])
    return cols


@pytest.mark.parametrize("name,L", [("lap", 256), ("st27", 512), ("rand", 128)])
def test_window_runs_expand_to_the_window(name, L):
    if name == "lap":
        n, _, rp, col, _ = synth.laplacian2d(60)
    elif name == "st27":
        n, _, rp, col, _ = synth.stencil27(12)
    else:
        n, _, rp, col, _ = synth.tiny_random(300, 2000, 0.01, 5)
    ti, tj = _aligned_tiles(rp, L)
    got = oracle.window_runs(tj, col)
    if name == "rand":  # scattered columns: far more than 14 runs per tile
        assert got is None
        return
    assert got is not None
    rec, codes = got
    t_of = _tile_of_each_nonzero(tj, len(col))
    for t in range(len(tj) - 1):
        cols = col[tj[t]:tj[t + 1]]
        window = sorted(set(int(c) for c in cols))      # brute force
        assert _expand_runs(rec[t]) == window
        # runs are maximal: consecutive runs are separated by a gap
        nr = int(rec[t, 1]) >> 16
        for r in range(nr - 1):
            end = (int(rec[t, 2 + r]) & 0xFFFF) + (int(rec[t, 2 + r]) >> 16)
            assert (int(rec[t, 3 + r]) & 0xFFFF) > end
    # the codes are the window ranks: the same as window codes
    assert np.array_equal(codes, oracle.window_codes(tj, col)[3])
    assert np.array_equal(np.array([_expand_runs(rec[t])[codes[j]] for j, t in enumerate(t_of)]), col)


def test_window_runs_laplacian_closed_form():
    # a tile of rows [a, b) of the 5-point Laplacian's grid interior has the
    # three bands [a-n, b-1-n], [a-1, b], [a+n, b-1+n] (b - a + 2 < n): three
    # runs of lengths b - a, b - a + 2, b - a starting at offsets 0, n - 1, 2n
    n = 100
    _, _, rp, col, _ = synth.laplacian2d(n)
    ti, tj = _aligned_tiles(rp, 256)
    rec, _ = oracle.window_runs(tj, col)
    checked = 0
    for t in range(len(tj) - 1):
        a, b = int(ti[t]), int(ti[t + 1])
        rows = np.arange(a, b)
        if b <= a or b - a + 2 >= n:
            continue
        x, y = rows % n, rows // n
        if x.min() < 1 or x.max() > n - 2 or y.min() < 1 or y.max() > n - 2:
            continue
        k = b - a
        assert list(rec[t, :5]) == [a - n, (3 * k + 2) | (3 << 16), 0 | (k << 16),
                                    (n - 1) | ((k + 2) << 16), (2 * n) | (k << 16)]
        checked += 1
    assert checked > 10


def test_window_runs_limits():
    def one_row(cols, max_runs=14):
        rp = np.array([0, len(cols)], dtype=np.int32)
        c = np.array(cols, dtype=np.int32)
        ti, tj = oracle.merge_tiles(rp, 1024, len(cols) + 1)
        return oracle.window_runs(tj, c, max_runs)
    # 14 runs fit, 15 do not (isolated columns: one run each)
    assert one_row(list(range(0, 28, 2))) is not None
    assert one_row(list(range(0, 30, 2))) is None
    # 256 consecutive columns are one run; 257 distinct do not fit the window
    rec, codes = one_row(list(range(1000, 1256)))
    assert list(rec[0, :3]) == [1000, 256 | (1 << 16), 0 | (256 << 16)]
    assert list(codes) == list(range(256))
    assert one_row(list(range(1000, 1257))) is None
    # range 2^16 - 1 fits, 2^16 does not
    assert one_row([3, 3 + 65535]) is not None
    assert one_row([3, 3 + 65536]) is None
    # repeated columns: one window entry, one code; an empty tile stays zero
    rec, codes = one_row([7, 8, 8, 7, 12, 13])
    assert list(rec[0, :4]) == [7, 4 | (2 << 16), 0 | (2 << 16), 5 | (2 << 16)]
    assert list(codes) == [0, 1, 1, 0, 2, 3]


# ------------------------------------------------------- SPD study matrices

def test_spd_generators_symmetric_and_dominant():
    """The amortization study's SPD systems: symmetric, positive diagonal,
    strictly diagonally dominant (27-point) or the Laplacian's weak
    dominance; the 7-point Laplacian has 7 s^3 - 6 s^2 nonzeros."""
    import scipy.sparse as sp
    for s in (5, 9):
        n, m, rp, col, val = synth.laplacian3d(s)
        assert len(col) == 7 * s ** 3 - 6 * s ** 2
        A = sp.csr_matrix((val, col, rp), shape=(n, m))
        assert (A - A.T).count_nonzero() == 0
        assert np.all(A.diagonal() == 6.0)
        n, m, rp, col, val = synth.spd_stencil27(s)
        A = sp.csr_matrix((val, col, rp), shape=(n, m))
        assert (A - A.T).count_nonzero() == 0
        d = A.diagonal()
        off = np.asarray(abs(A).sum(axis=1)).ravel() - d
        assert np.all(d > off)
        assert np.all(d >= 1.0)


def test_localized_irregular_generator():
    """The partition study's matrices: 16 sorted distinct columns in every
    row; outside the stretch [n/2, n/2 + f n) each row is the contiguous
    window starting at i - 8 (shifted inside [0, n)), inside it the columns
    are spread (not one window)."""
    n = 4096
    for frac in (0.0, 1 / 64, 1 / 4):
        n_, m, rp, col, val = synth.localized_irregular(n, 16, frac, 811)
        assert n_ == m == n and np.array_equal(rp, np.arange(n + 1) * 16)
        c = col.reshape(n, 16).astype(np.int64)
        assert np.all(np.diff(c, axis=1) > 0) and c.min() >= 0 and c.max() < n
        r0, r1 = n // 2, n // 2 + round(frac * n)
        start = np.clip(np.arange(n) - 8, 0, n - 16)
        regular = np.ones(n, dtype=bool)
        regular[r0:r1] = False
        assert np.array_equal(c[regular], (start[:, None] + np.arange(16))[regular])
        if r1 > r0:
            assert np.all(c[r0:r1, -1] - c[r0:r1, 0] > 16)
        assert np.all((val > 0) & (val <= 1))


# ------------------------------------------------------------ column blocks

@pytest.mark.parametrize("B", [1, 2, 3, 4, 8])
def test_column_blocks_partition_in_storage_order(B):
    n, m, rp, col, val = synth.tiny_random(500, 997, 0.02, 31)
    width = (m + B - 1) // B
    rpb, colb, valb = oracle.column_blocks(rp, col, val, B, width)
    rows = np.repeat(np.arange(n), np.diff(rp))
    off = 0
    got = []
    for b in range(B):
        r = rpb[b]
        assert r[0] == 0 and np.all(np.diff(r) >= 0)
        k = int(r[-1])
        cb, vb = colb[off:off + k], valb[off:off + k]
        assert np.all((cb >= b * width) & (cb < (b + 1) * width))
        for i in range(n):
            # the block's part of row i is the row's in-block entries, in order
            sel = (col[rp[i]:rp[i + 1]] >= b * width) & (col[rp[i]:rp[i + 1]] < (b + 1) * width)
            assert np.array_equal(cb[r[i]:r[i + 1]], col[rp[i]:rp[i + 1]][sel])
            assert np.array_equal(vb[r[i]:r[i + 1]], val[rp[i]:rp[i + 1]][sel])
        got.append(k)
        off += k
    assert off == len(col)                      # every nonzero exactly once
    if B == 1:
        assert np.array_equal(rpb[0], rp) and np.array_equal(colb, col)


def test_column_blocks_sum_to_the_product():
    """y = sum over blocks of the block products, in block order: bit-exact on
    dyadic inputs (every partial sum exact)."""
    n, m, rp, col, val = synth.tiny_random(400, 640, 0.05, 33, dyadic=True)
    x = synth.dyadic_vector(m, 5)
    for B in (2, 5):
        width = (m + B - 1) // B
        rpb, colb, valb = oracle.column_blocks(rp, col, val, B, width)
        y = np.zeros(n)
        off = 0
        for b in range(B):
            k = int(rpb[b][-1])
            y = y + oracle.spmv(rpb[b], colb[off:off + k], valb[off:off + k], x)
            off += k
        assert np.array_equal(y, oracle.spmv(rp, col, val, x))


def test_column_block_rows_by_brute_force():
    """Row lists of blocks 1 .. B-1: the rows with a nonzero whose column lies
    in the block (Python sets over the CSR itself), ascending, with row
    pointers counting those nonzeros; and the block products through the
    lists add up to the product (dyadic inputs, bit-exact)."""
    n, m, rp, col, val = synth.tiny_random(300, 900, 0.01, 35, dyadic=True)
    x = synth.dyadic_vector(m, 7)
    for B in (2, 3, 8):
        width = (m + B - 1) // B
        rpb, colb, valb = oracle.column_blocks(rp, col, val, B, width)
        rows, ptr = oracle.column_block_rows(rpb)
        ro = po = 0
        y = oracle.spmv(rpb[0], colb[:rpb[0][-1]], valb[:rpb[0][-1]], x)
        off = int(rpb[0][-1])
        for b in range(1, B):
            want = sorted({i for i in range(n) for j in range(rp[i], rp[i + 1])
                           if b * width <= col[j] < (b + 1) * width})
            k = len(want)
            assert list(rows[ro:ro + k]) == want
            p = ptr[po:po + k + 1]
            assert p[0] == 0
            counts = [sum(1 for j in range(rp[i], rp[i + 1]) if b * width <= col[j] < (b + 1) * width)
                      for i in want]
            assert list(np.diff(p)) == counts
            nb = int(p[-1])
            part = oracle.spmv(p, colb[off:off + nb], valb[off:off + nb], x)
            y[want] = y[want] + part
            off += nb
            ro += k
            po += k + 1
        assert ro == rows.size and po == ptr.size
        if B == 8:  # rows without nonzeros in some blocks are left out
            assert rows.size < (B - 1) * n
        assert np.array_equal(y, oracle.spmv(rp, col, val, x))


def test_window_codes_nine_bit_ranks_by_brute_force():
    """Windows of up to 512 entries (9-bit ranks on tiles of 1,024 items):
    the ranks are the positions in the sorted set of the tile's columns
    (Python sets), 512 distinct columns fit and 513 do not, and the
    ninth-bit records put rank >= 256 at the lane and bit that load the
    element (walking the lanes' load order element by element)."""
    n = 3000
    # tridiagonal-like rows: about 256 rows and 258 distinct columns per tile
    rows = np.repeat(np.arange(n), 3)
    cols = np.clip(rows + np.tile([-1, 0, 1], n), 0, n - 1)
    keep = np.ones(rows.size, bool)
    keep[[0, rows.size - 1]] = False  # row 0 and row n-1 have two entries
    rows, cols = rows[keep], cols[keep]
    rp = np.searchsorted(rows, np.arange(n + 1)).astype(np.int32)
    col = cols.astype(np.int32)
    ti, tj = _aligned_tiles(rp, 1024)
    base, wlen, dct, ranks = oracle.window_codes(tj, col, 512)
    assert ranks.dtype == np.uint16 and ranks.max() >= 256
    for t in range(len(tj) - 1):
        c = col[tj[t]:tj[t + 1]]
        u = sorted(set(int(v) for v in c))
        assert wlen[t] == len(u) and (not u or base[t] == u[0])
        assert [int(v) for v in ranks[tj[t]:tj[t + 1]]] == [u.index(int(v)) for v in c]
        assert [int(v) for v in dct[t, :len(u)]] == [v - u[0] for v in u]
    assert oracle.window_codes(tj, col, 256) is None  # more than 256 distinct in a tile
    for vec in (2, 4):
        rec = oracle.window_rank_records(tj, ranks, wlen, vec)
        masks = rec[:, 1:].view(np.uint16).reshape(len(tj) - 1, 64)
        assert np.array_equal(rec[:, 0], wlen)
        for t in range(len(tj) - 1):
            for lane in range(64):
                for it in range(1024 // (64 * vec)):
                    for e in range(vec):
                        p = it * 64 * vec + lane * vec + e
                        bit = (int(masks[t, lane]) >> (it * vec + e)) & 1
                        want = p < tj[t + 1] - tj[t] and ranks[tj[t] + p] >= 256
                        assert bit == int(want), (t, lane, it, e)
    # 512 distinct columns fit, 513 do not
    one = lambda k: oracle.window_codes(np.array([0, k], np.int32), np.arange(k, dtype=np.int32) * 3, 512)
    assert one(512) is not None and one(513) is None

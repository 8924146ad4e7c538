"""Degenerate and boundary shapes through every path: all rows empty, a 1 x 1
matrix, one dense row, one column, only the last row filled, unsorted rows
with repeated columns, rows of 62-65 and 60-63 nonzeros (either side of the
row-aligned tiles' limit), N + NNZ exactly one tile and one item past it,
and banded rows whose windows need 9-bit ranks or fit neither window width.
Every catalogue variant at every prebuilt tile size, the selectors, the
batched launch and the allocation-free entry point. Values are small
integers and x is dyadic, so FP64 results must equal the oracle's bit for
bit (Sec. II, Fig. 2); FP32/BF16 storage is held to its a-priori bound.
Rows without nonzeros must give +0.0."""
import numpy as np
import pytest
import torch

import oracle
import paper_1711_05487_amd as pkg
import synth
from paper_1711_05487_amd import learn, tree
from spmv_cases import check_reduced

pytestmark = pytest.mark.gpu

MERGE = pkg.OPT_MERGE


def dyadic_values(nnz, seed):
    v = (synth.uindex(seed, 1, np.arange(nnz, dtype=np.uint64), 17) - 8).astype(np.float64)
    v[v == 0] = 1.0
    return v


def from_lengths(lens, m, seed):
    """Rows of the given lengths with distinct sorted columns in [0, m)."""
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    cols = []
    for i, l in enumerate(lens):
        if l == 0:
            continue
        if l == m:
            cols.append(np.arange(m))
            continue
        c = np.unique(synth.uindex(seed, 2 + i, np.arange(4 * l, dtype=np.uint64), m))[:l]
        assert c.size == l, (i, l)
        cols.append(c)
    col = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, dtype=np.int32)
    return rp, col


def shapes():
    out = {}
    out["all rows empty"] = (3, 4, np.zeros(4, dtype=np.int32), np.zeros(0, dtype=np.int32))
    out["1 x 1"] = (1, 1, np.array([0, 1], dtype=np.int32), np.array([0], dtype=np.int32))
    out["one dense row"] = (1, 5000, np.array([0, 5000], dtype=np.int32),
                            np.arange(5000, dtype=np.int32))
    out["one column"] = (5000, 1, np.arange(5001, dtype=np.int32), np.zeros(5000, dtype=np.int32))
    lens = [0] * 1999 + [300]
    out["only the last row"] = (2000, 2000) + from_lengths(lens, 2000, 31)
    lens = [60, 61, 62, 63] * 100  # the longest rows that still give row-aligned tiles
    out["rows of 60-63"] = (400, 1000) + from_lengths(lens, 1000, 38)
    lens = [62, 63, 64, 65] * 100
    out["rows of 62-65"] = (400, 1000) + from_lengths(lens, 1000, 32)
    # rows of 64 or more nonzeros: tiles cut every L items, so N + NNZ =
    # 1,024 is one tile of 1,024 items exactly, and 1,025 one item past it
    lens = [127] * 8
    out["one tile exactly"] = (8, 300) + from_lengths(lens, 300, 33)
    lens = [127] * 7 + [128]
    out["one item past a tile"] = (8, 300) + from_lengths(lens, 300, 34)
    # unsorted rows with repeated columns (summed in storage order; delta
    # codes need sorted rows and must not be built)
    lens = synth.uindex(39, 0, np.arange(300, dtype=np.uint64), 41)
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    col = synth.uindex(39, 1, np.arange(rp[-1], dtype=np.uint64), 60).astype(np.int32)
    out["unsorted, repeated columns"] = (300, 60, rp, col)
    for bw in (200, 700):  # windows of 9-bit ranks / of neither width
        n, m, rp, col, _ = synth.banded_random(4000, bw, 16, 35)
        out[f"band {bw}"] = (n, m, rp, col)
    return out


SHAPES = shapes()


def variants():
    for opts in oracle.catalogue():
        if opts & MERGE:
            for L in (0, 256, 512, 1024):
                yield {"mode": "forced", "forced_opts": opts, "merge_items": L}
        else:
            yield {"mode": "forced", "forced_opts": opts}
    for mode in ("plain", "profile", "learned", "tree"):
        yield {"mode": mode}
    yield {"mode": "exhaustive", "timing_calls": 2}


@pytest.fixture(scope="module", autouse=True)
def models():
    learn.install()
    tree.install()


def run(A, x32):
    xd = torch.from_numpy(np.ascontiguousarray(x32)).cuda()
    y = A.spmv(xd)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def check(y, rp, col, val, x, storage, what):
    empty = np.diff(rp) == 0
    assert not np.signbit(y[empty]).any(), f"{what}: -0.0 in an empty row"
    if storage == "f64":
        want = oracle.spmv(rp, col, val, x)
        assert np.array_equal(y, want), f"{what}: rows {np.nonzero(y != want)[0][:5]}"
    else:
        check_reduced(y, rp, col, val, x, storage, what)


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("name", list(SHAPES))
def test_every_variant(name, storage):
    n, m, rp, col = SHAPES[name]
    val = dyadic_values(col.size, 36)
    x = synth.dyadic_vector(m, 37)
    xin = x if storage == "f64" else oracle.to_f32(x)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m, storage=storage)
    try:
        check(run(A, xin), rp, col, val, x, storage, f"{name} {storage} before any selection")
        for v in variants():
            kw = dict(v)
            info = A.select(kw.pop("mode"), **kw)
            what = f"{name} {storage} {v} -> opts {info['opts']} L {info['merge_items']}"
            check(run(A, xin), rp, col, val, x, storage, what)
    finally:
        A.close()


def test_unsorted_rows_get_no_delta_codes():
    n, m, rp, col = SHAPES["unsorted, repeated columns"]
    assert not oracle.rows_sorted(rp, col)
    A = pkg.CsrMatrix(rp, col, dyadic_values(col.size, 36), n_cols=m)
    assert A.select("forced", forced_opts=pkg.OPT_DELTA)["delta_bits"] == 32
    A.close()


def test_nine_bit_and_fallback_windows_chosen():
    """The two banded shapes reach the window paths they are here for: 9-bit
    ranks on 1,024-item tiles, and (windows too wide for either width) the
    tile-base codes on 512-item tiles."""
    got = {}
    for bw in (200, 700):
        n, m, rp, col = SHAPES[f"band {bw}"]
        A = pkg.CsrMatrix(rp, col, dyadic_values(col.size, 36), n_cols=m)
        info = A.select("forced", forced_opts=MERGE | pkg.OPT_DELTA)
        got[bw] = (info["merge_items"], info["window_codes"], info["delta_bits"])
        A.close()
    assert got[200] == (1024, 3, 9), got
    assert got[700][0] == 512 and got[700][1] == 0 and got[700][2] == 16, got


@pytest.mark.parametrize("storage", ["f64", "bf16"])
def test_batched_degenerate_shapes(storage):
    """Every shape in one batched launch (plus a matrix without rows), each
    with its learned plan and again with forced merge tiles: every y equals
    the matrix's own csr_spmv bit for bit."""
    hs, xs, ys, own = [], [], [], []
    dt = torch.float64 if storage == "f64" else torch.float32
    try:
        for k, (name, (n, m, rp, col)) in enumerate(SHAPES.items()):
            A = pkg.CsrMatrix(rp, col, dyadic_values(col.size, 40 + k), n_cols=m, storage=storage)
            hs.append(A)
            x = synth.dyadic_vector(m, 60 + k)
            xs.append(torch.from_numpy(x if storage == "f64" else oracle.to_f32(x)).cuda())
        E = pkg.CsrMatrix(np.zeros(1, dtype=np.int32), np.zeros(0, dtype=np.int32), np.zeros(0),
                          n_cols=3, storage=storage)
        hs.append(E)
        xs.append(torch.ones(3, dtype=dt, device="cuda"))
        for sel in ({"mode": "learned"}, {"mode": "forced", "forced_opts": MERGE | pkg.OPT_DELTA}):
            own.clear()
            ys.clear()
            for A, x in zip(hs, xs):
                kw = dict(sel)
                A.select(kw.pop("mode"), **kw)
                own.append(A.spmv(x).clone() if A.n_rows > 0 else None)
                ys.append(torch.full((max(A.n_rows, 1),), 7.0, dtype=dt, device="cuda")[:A.n_rows])
            pkg.spmv_batched(hs, xs, ys)
            torch.cuda.synchronize()
            for k, (y, ref) in enumerate(zip(ys, own)):
                if ref is not None:
                    assert torch.equal(y, ref), (sel, k)
    finally:
        for A in hs:
            A.close()


@pytest.mark.parametrize("name", list(SHAPES))
def test_noalloc_degenerate_shapes(name):
    n, m, rp, col = SHAPES[name]
    val = dyadic_values(col.size, 36)
    x = synth.dyadic_vector(m, 37)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    y = torch.full((n,), 5.0, dtype=torch.float64, device="cuda")
    pkg.spmv_noalloc(n, m, t(rp), t(col), t(val), t(x), y)
    torch.cuda.synchronize()
    check(y.cpu().numpy(), rp, col, val, x, "f64", f"noalloc {name}")

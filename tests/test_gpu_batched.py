"""GPU parity of csr_spmv_batched (one graph-captured launch over many
matrices, each running its own plan): bit-identical to each matrix's own
csr_spmv for every catalogue variant and for learned plans, within the FP64
bar against the oracle, stable across graph replays interleaved with eager
work, and correct when back-to-back calls move the vectors."""
import numpy as np
import pytest
import torch

import oracle
import paper_1711_05487_amd as pkg
import synth
from spmv_cases import check_f64, check_reduced

pytestmark = pytest.mark.gpu


def batch_mats(count, storage="f64", with_empty=True):
    mats = [synth.batch_matrix(i)[1] for i in range(count)]
    if with_empty:
        mats.append((7, 5, np.zeros(8, dtype=np.int32), np.zeros(0, dtype=np.int32), np.zeros(0)))
        mats.append(synth.tiny_random(40, 30, 0.3, 3))
    hs = [pkg.CsrMatrix(rp, col, val, n_cols=m, storage=storage) for (n, m, rp, col, val) in mats]
    return mats, hs


def vectors(mats, seed, dtype=torch.float64):
    xs = [torch.from_numpy(synth.vector(m, seed + k)).to(dtype).cuda() for k, (n, m, *_ ) in enumerate(mats)]
    ys = [torch.full((max(n, 1),), float("nan"), dtype=dtype, device="cuda") for (n, *_ ) in mats]
    return xs, ys


def test_batched_bit_identical_to_single_merge():
    mats, hs = batch_mats(24)
    for k, A in enumerate(hs):  # each matrix keeps its own tile size
        A.select("forced", forced_opts=pkg.OPT_MERGE, merge_items=(256, 512, 1024)[k % 3])
    xs, ys = vectors(mats, 100)
    pkg.spmv_batched(hs, xs, ys)
    torch.cuda.synchronize()
    for k, A in enumerate(hs):
        single = A.spmv(xs[k])
        torch.cuda.synchronize()
        n = mats[k][0]
        assert torch.equal(ys[k][:n], single[:n]), k


def test_batched_bit_identical_to_single_merge_codes():
    """Merge codes and window codes (MERGE|DELTA): the batch reads the same
    codes with the same tiles as the single launches, so the same bits."""
    mats, hs = batch_mats(12)
    for k, A in enumerate(hs):
        A.select("forced", forced_opts=pkg.OPT_MERGE | pkg.OPT_DELTA, merge_items=(256, 512)[k % 2])
    xs, ys = vectors(mats, 150)
    pkg.spmv_batched(hs, xs, ys)
    torch.cuda.synchronize()
    for k, A in enumerate(hs):
        single = A.spmv(xs[k])
        torch.cuda.synchronize()
        n = mats[k][0]
        assert torch.equal(ys[k][:n], single[:n]), k


def test_batched_autotuned_matches_oracle_and_replays():
    mats, hs = batch_mats(40)
    eager = None
    for rep in range(4):
        xs, ys = vectors(mats, 200 + rep)   # new vector pointers every call
        pkg.spmv_batched(hs, xs, ys)
        torch.cuda.synchronize()
        # eager work between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        for k, (n, m, rp, col, val) in enumerate(mats):
            check_f64(ys[k][:n].cpu().numpy(), rp, col, val, xs[k].cpu().numpy(), f"batch {k} rep {rep}")
        if rep == 0:
            eager = [y.clone() for y in ys]
            x0 = xs
        assert junk.isfinite()
    # replay with the first call's vectors: identical bits
    ys = [torch.empty_like(y) for y in eager]
    pkg.spmv_batched(hs, x0, ys)
    torch.cuda.synchronize()
    for k, (n, *_ ) in enumerate(mats):
        assert torch.equal(ys[k][:n], eager[k][:n])


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_batched_reduced_precision(storage):
    mats, hs = batch_mats(12, storage=storage)
    xs64 = [synth.vector(m, 300 + k) for k, (n, m, *_ ) in enumerate(mats)]
    xs = [torch.from_numpy(oracle.to_f32(x)).cuda() for x in xs64]
    ys = [torch.empty(max(n, 1), dtype=torch.float32, device="cuda") for (n, *_ ) in mats]
    pkg.spmv_batched(hs, xs, ys)
    torch.cuda.synchronize()
    for k, (n, m, rp, col, val) in enumerate(mats):
        check_reduced(ys[k][:n].cpu().numpy(), rp, col, val, xs64[k], storage, f"batch {k}")


def test_batched_dyadic_exact():
    mats = [synth.tiny_random(300 + 37 * k, 200, 0.05 + 0.02 * k, 40 + k, dyadic=True) for k in range(10)]
    hs = [pkg.CsrMatrix(rp, col, val, n_cols=m) for (n, m, rp, col, val) in mats]
    xs = [torch.from_numpy(synth.dyadic_vector(m, 50 + k)).cuda() for k, (n, m, *_ ) in enumerate(mats)]
    ys = [torch.empty(n, dtype=torch.float64, device="cuda") for (n, *_ ) in mats]
    pkg.spmv_batched(hs, xs, ys)
    torch.cuda.synchronize()
    for k, (n, m, rp, col, val) in enumerate(mats):
        assert np.array_equal(ys[k].cpu().numpy(), oracle.spmv(rp, col, val, xs[k].cpu().numpy()))


def test_batched_errors_and_handle_lifetime():
    a = synth.tiny_random(50, 50, 0.1, 1)
    b = synth.tiny_random(60, 50, 0.1, 2)
    A = pkg.CsrMatrix(a[2], a[3], a[4], n_cols=50)
    B32 = pkg.CsrMatrix(b[2], b[3], b[4], n_cols=50, storage="f32")
    x = torch.ones(50, dtype=torch.float64, device="cuda")
    y = torch.empty(60, dtype=torch.float64, device="cuda")
    with pytest.raises(pkg.CsrError):
        pkg.spmv_batched([A, B32], [x, x.float()], [y, y.float()])   # mixed storage
    B = pkg.CsrMatrix(b[2], b[3], b[4], n_cols=50)
    pkg.spmv_batched([A, B], [x, x], [y[:50], y])
    torch.cuda.synchronize()
    B.close()  # drops the cached plan
    C = pkg.CsrMatrix(b[2], b[3], b[4], n_cols=50)
    y2 = torch.empty(60, dtype=torch.float64, device="cuda")
    pkg.spmv_batched([A, C], [x, x], [torch.empty(50, dtype=torch.float64, device="cuda"), y2])
    torch.cuda.synchronize()
    check_f64(y2.cpu().numpy(), b[2], b[3], b[4], np.ones(50), "after destroy")


def same_as_single(mats, hs, xs, ys, what):
    for k, A in enumerate(hs):
        single = A.spmv(xs[k])
        torch.cuda.synchronize()
        n = mats[k][0]
        assert torch.equal(ys[k][:n], single[:n]), f"{what}: matrix {k}"


def test_batched_every_catalogue_variant_bit_identical():
    """Every variant of the 16-entry catalogue (row split with delta codes,
    streaming, unrolling and long rows; merge tiles with codes, window codes
    and column blocks), several matrices per variant and several variants
    per batch, each bit-identical to its own csr_spmv and within the FP64 bar."""
    cat = [0, 1, 2, 4, 8, 16] + [a | b for i, a in enumerate((1, 2, 4, 8, 16))
                                 for b in (1, 2, 4, 8, 16)[i + 1:]]
    mats = [synth.batch_matrix(i)[1] for i in range(32)]
    mats.append(synth.stencil27(10))
    mats.append(synth.uniform_random(600_000, 8))     # x beyond an L2: column blocks (P|M)
    mats.append(synth.rmat(12, 16))                   # long rows: decomposition (D|X)
    mats.append(synth.stencil27(12))                  # short rows: window codes (D|M)
    hs = [pkg.CsrMatrix(rp, col, val, n_cols=m) for (n, m, rp, col, val) in mats]
    xs, ys = vectors(mats, 400)
    seen = set()
    for shift in range(4):
        for k, A in enumerate(hs):
            info = A.select("forced", forced_opts=cat[(k + 5 * shift) % 16], long_row_floor=256,
                            long_row_factor=8.0, dynamic_rows=k % 2)
            seen.add((info["opts"], info["window_codes"], info["column_blocks"] > 1,
                      info["n_long_rows"] > 0))
        pkg.spmv_batched(hs, xs, ys)
        torch.cuda.synchronize()
        same_as_single(mats, hs, xs, ys, f"shift {shift}")
        for k, (n, m, rp, col, val) in enumerate(mats):
            check_f64(ys[k][:n].cpu().numpy(), rp, col, val, xs[k].cpu().numpy(), f"batch {k}")
    assert any(w for _, w, _, _ in seen) and any(c for _, _, c, _ in seen)
    assert any(l for *_, l in seen)


def test_batched_learned_plans_bit_identical():
    from paper_1711_05487_amd import learn
    learn.install()
    mats = [synth.batch_matrix(i)[1] for i in range(64)]
    hs = [pkg.CsrMatrix(rp, col, val, n_cols=m) for (n, m, rp, col, val) in mats]
    opts = set()
    for A in hs:
        opts.add(A.select("learned")["opts"])
    assert len(opts) >= 3
    xs, ys = vectors(mats, 500)
    pkg.spmv_batched(hs, xs, ys)
    torch.cuda.synchronize()
    same_as_single(mats, hs, xs, ys, "learned")


def test_batched_full_512_matrix_set_matches_oracle():
    """The benchmark's 512-matrix batch (1,024-65,536 rows, every suite
    family), each matrix with its learned plan: every y within the FP64 bar
    against the oracle and bit-identical to the matrix's own csr_spmv, and a
    second call with the same vectors replays the same bits."""
    from paper_1711_05487_amd import learn
    learn.install()
    mats = [synth.batch_matrix(i)[1] for i in range(512)]
    hs = [pkg.CsrMatrix(rp, col, val, n_cols=m) for (n, m, rp, col, val) in mats]
    try:
        for A in hs:
            A.select("learned")
        xs, ys = vectors(mats, 602)
        pkg.spmv_batched(hs, xs, ys)
        torch.cuda.synchronize()
        first = [y.clone() for y in ys]
        for k, (n, m, rp, col, val) in enumerate(mats):
            check_f64(ys[k][:n].cpu().numpy(), rp, col, val, xs[k].cpu().numpy(), f"C5 matrix {k}")
        same_as_single(mats, hs, xs, ys, "C5 learned")
        pkg.spmv_batched(hs, xs, ys)
        torch.cuda.synchronize()
        for k, (n, *_ ) in enumerate(mats):
            assert torch.equal(ys[k][:n], first[k][:n]), f"C5 replay {k}"
    finally:
        for A in hs:
            A.close()


def test_batched_back_to_back_moving_vectors():
    """Calls issued without waiting, each with new vectors: the descriptor
    refresh of one call must not change what the previous call reads."""
    mats, hs = batch_mats(20)
    for k, A in enumerate(hs):
        A.select("forced", forced_opts=(0, 1, 8, 9, 16)[k % 5])
    sets = [vectors(mats, 600 + 10 * r) for r in range(4)]
    for xs, ys in sets:
        pkg.spmv_batched(hs, xs, ys)
    torch.cuda.synchronize()
    for r, (xs, ys) in enumerate(sets):
        for k, (n, m, rp, col, val) in enumerate(mats):
            check_f64(ys[k][:n].cpu().numpy(), rp, col, val, xs[k].cpu().numpy(),
                      f"call {r} matrix {k}")


def test_batched_column_blocks_with_split_rows():
    """Column-blocked merge plans on tiles that are not row-aligned (R-MAT
    scale 21: every pass with its carries and fixup) beside row-aligned
    column blocks and small plans: bit-identical to each matrix's own
    csr_spmv, within the FP64 bar, and the same on a replay."""
    mats = [synth.rmat(21, 16), synth.uniform_random(600_000, 8)]
    mats += [synth.batch_matrix(i)[1] for i in range(6)]
    hs = [pkg.CsrMatrix(rp, col, val, n_cols=m) for (n, m, rp, col, val) in mats]
    for k, A in enumerate(hs):
        info = A.select("forced", forced_opts=pkg.OPT_MERGE, split_row_blocks=1)
        if k == 0:
            assert info["column_blocks"] == 8 and info["merge_slack"] == 0
        if k == 1:
            assert info["column_blocks"] == 3 and info["merge_slack"] > 0
    xs, ys = vectors(mats, 700)
    pkg.spmv_batched(hs, xs, ys)
    torch.cuda.synchronize()
    first = [y.clone() for y in ys]
    same_as_single(mats, hs, xs, ys, "split-row column blocks")
    for k, (n, m, rp, col, val) in enumerate(mats):
        check_f64(first[k][:n].cpu().numpy(), rp, col, val, xs[k].cpu().numpy(), f"batch {k}")
    pkg.spmv_batched(hs, xs, ys)
    torch.cuda.synchronize()
    for k, (n, *_ ) in enumerate(mats):
        assert torch.equal(ys[k][:n], first[k][:n]), k


def test_batched_nine_bit_windows_bit_identical():
    """9-bit window ranks (1,024-item tiles) beside 8-bit windows and other
    plans in one batch: the same bits as each matrix's own csr_spmv."""
    n0, m0, rp0, col0, val0 = synth.stencil27(24)
    mats = [(n0, m0, rp0, col0, val0), synth.stencil27(20)]
    mats += [synth.batch_matrix(i)[1] for i in range(6)]
    hs = [pkg.CsrMatrix(rp, col, val, n_cols=m) for (n, m, rp, col, val) in mats]
    for k, A in enumerate(hs):
        info = A.select("forced", forced_opts=pkg.OPT_MERGE | pkg.OPT_DELTA,
                        merge_items=1024 if k < 2 else 512)
        if k < 2:
            assert info["window_codes"] == 3
    xs, ys = vectors(mats, 800)
    pkg.spmv_batched(hs, xs, ys)
    torch.cuda.synchronize()
    same_as_single(mats, hs, xs, ys, "9-bit windows")
    for k, (n, m, rp, col, val) in enumerate(mats):
        check_f64(ys[k][:n].cpu().numpy(), rp, col, val, xs[k].cpu().numpy(), f"batch {k}")

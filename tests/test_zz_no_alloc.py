"""csr_spmv_noalloc, the entry point for callers that cannot allocate: its
result against csr_spmv with the same kernel and schedule (forced plain plan
with dynamic row chunks), bit for bit, on two calls in a row (the second on
a smaller matrix, so stale counter or scratch contents would show), and
against the oracle at the FP64 bar."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1711_05487_amd as pkg
import synth
from spmv_cases import check_f64, matrix

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def reference(n, m, rp, col, val, x):
    """The existing entry point: csr_spmv on a handle with the same plan."""
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    info = A.select("forced", forced_opts=0, dynamic_rows=1)
    assert info["dynamic_rows"] == 1 and info["opts"] == 0
    y = A.spmv(dev(x))
    torch.cuda.synchronize()
    A.close()
    return y.cpu().numpy()


def no_alloc(n, m, rp, col, val, x):
    y = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
    pkg.spmv_noalloc(n, m, dev(rp), dev(col), dev(val), dev(x), y)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def test_noalloc_matches_csr_spmv_on_two_calls():
    cases = [("rmat14", matrix("rmat14")), ("lap37", matrix("lap37"))]
    for k, (name, (n, m, rp, col, val)) in enumerate(cases):
        x = synth.vector(m, 77 + k)
        got = no_alloc(n, m, rp, col, val, x)
        ref = reference(n, m, rp, col, val, x)
        assert np.array_equal(got, ref), name
        check_f64(got, rp, col, val, x, f"noalloc {name}")


def test_noalloc_rectangular_and_empty_rows():
    n, m, rp, col, val = synth.tiny_random(700, 333, 0.03, 5)
    lens = np.diff(rp)
    lens[::7] = 0  # every seventh row emptied
    keep = np.repeat(lens > 0, np.diff(rp))
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    col, val = col[keep], val[keep]
    x = synth.vector(m, 6)
    got = no_alloc(n, m, rp, col, val, x)
    assert np.array_equal(got, reference(n, m, rp, col, val, x))
    check_f64(got, rp, col, val, x, "noalloc rectangular")


def test_noalloc_rejects_bad_arguments():
    L = pkg.lib()
    P = ctypes.c_void_p
    assert L.csr_spmv_noalloc(-1, 4, 0, P(8), None, None, P(8), P(64), None) == 1
    assert L.csr_spmv_noalloc(4, 4, 8, P(8), None, P(8), P(8), P(64), None) == 1
    assert L.csr_spmv_noalloc(4, 4, 1 << 31, P(8), P(8), P(8), P(8), P(64), None) == 5
    # x and y overlapping
    assert L.csr_spmv_noalloc(4, 4, 4, P(8), P(8), P(8), P(4096), P(4096 + 8), None) == 1
    assert b"overlap" in L.csr_last_error()
    # an empty matrix is a no-op
    assert L.csr_spmv_noalloc(0, 0, 0, P(8), None, None, None, None, None) == 0

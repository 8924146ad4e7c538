"""The conjugate-gradient harness of the amortization study (bench.py
--amortize) on small SPD systems: the solution it reaches with each
optimizer's plan agrees with a dense solve, and every plan takes the same
number of iterations within one residual check."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import bench
import paper_1711_05487_amd as pkg
import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("gen", [lambda: synth.laplacian3d(12), lambda: synth.spd_stencil27(10),
                                 lambda: synth.laplacian2d(40)])
def test_pcg_converges_with_every_plan(gen):
    n, m, rp, col, val = gen()
    x_true = synth.vector(m, 901)
    dense = sp.csr_matrix((val, col, rp), shape=(n, m)).toarray()
    b_np = dense @ x_true
    diag = np.diag(dense).copy()
    b = torch.from_numpy(b_np).cuda()
    dinv = torch.from_numpy(1.0 / diag).cuda()
    its = []
    for lab, mode, over in bench.OPTIMIZERS:
        A = pkg.CsrMatrix(rp, col, val, n_cols=m)
        A.select(mode, timing_calls=8, **over)
        xs, it = bench.pcg(A, b, dinv, tol=1e-10)
        torch.cuda.synchronize()
        got = xs.cpu().numpy()
        assert np.linalg.norm(got - x_true) <= 1e-7 * np.linalg.norm(x_true), lab
        its.append(it)
        A.close()
    assert max(its) - min(its) <= 8, its

"""Selection by the feature-guided classifier (CSR_SEL_TREE): the library
walks the committed tree on its own features and applies the Table II
remedies of the predicted classes; without a tree it falls back to the
profile-guided path."""
import numpy as np
import pytest
import torch

import oracle
import paper_1711_05487_amd as pkg
from paper_1711_05487_amd import tree
from spmv_cases import check_f64, matrix, xvec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def committed_tree():
    tree.install()
    yield
    pkg.tree_unload()


@pytest.mark.parametrize("name", ["lap100", "st27_24", "rmat14", "unif14"])
def test_tree_selection_follows_the_tree(name):
    n, m, rp, col, val = matrix(name)
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    info = A.select("tree")
    f, _, _ = A.inspect()
    cls = int(tree.predict(tree.load(), f[None, :])[0])
    assert info["fallback"] == 0
    assert info["classes"] == cls
    tau = int(max(32.0 * f[3], 4096))  # default long-row threshold of the library
    assert info["opts"] == oracle.remedies(cls, f[2] > tau, pkg.default_config().remedy_map)
    x = xvec(name, m)
    y = A.spmv(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    check_f64(y.cpu().numpy(), rp, col, val, x, f"{name} tree")
    A.close()


def test_tree_selection_falls_back_without_a_tree():
    n, m, rp, col, val = matrix("st27_24")
    A = pkg.CsrMatrix(rp, col, val, n_cols=m)
    pkg.tree_unload()
    try:
        info = A.select("tree", timing_calls=8)
        assert info["fallback"] == 1 and info["classes"] >= 0
    finally:
        tree.install()
    assert A.select("tree")["fallback"] == 0
    A.close()

"""The feature-guided classifier's CART (Sec. III-D) on the host: the split it
picks against a brute-force search and against scikit-learn's tree, the match
ratios of Sec. IV-B on hand-made cases, the committed tree, and the ABI's
checks of a tree handed to the library (host-only calls)."""
import itertools
import json
import os

import numpy as np
import pytest

import paper_1711_05487_amd as pkg
from paper_1711_05487_amd import learn, tree
import synth


def _data(n, f, seed, bits=4):
    X = synth.u01(seed, 0, np.arange(n * f, dtype=np.uint64)).reshape(n, f)
    y = synth.uindex(seed, 1, np.arange(n, dtype=np.uint64), 1 << bits).astype(np.int64)
    return X, y


def _gini_bits(Y):
    p = Y.mean(axis=0)
    return np.mean(1 - p ** 2 - (1 - p) ** 2)


def test_root_split_is_the_brute_force_best():
    for seed in (3, 4, 5):
        X, y = _data(36, 3, seed)
        Y = tree.masks_to_bits(y)
        best = None
        for f in range(3):
            vals = sorted(set(X[:, f]))
            for a, b in zip(vals, vals[1:]):
                thr = (a + b) / 2
                L, R = Y[X[:, f] <= thr], Y[X[:, f] > thr]
                if len(L) < 2 or len(R) < 2:
                    continue
                dec = len(Y) * _gini_bits(Y) - len(L) * _gini_bits(L) - len(R) * _gini_bits(R)
                if best is None or dec > best[0] + 1e-12:
                    best = (dec, f, thr)
        f, thr = tree.best_split(X, Y, min_leaf=2)
        assert (f, thr) == (best[1], best[2])


def test_root_split_matches_scikit_learn():
    from sklearn.tree import DecisionTreeClassifier
    for seed in (11, 12, 13, 14):
        X, y = _data(200, 6, seed)
        Y = tree.masks_to_bits(y)
        sk = DecisionTreeClassifier(criterion="gini", max_depth=1, random_state=0).fit(X, Y)
        f, thr = tree.best_split(X, Y, min_leaf=1)
        assert f == sk.tree_.feature[0]
        # scikit-learn splits a float32 copy of X: thresholds agree to float32
        assert thr == pytest.approx(sk.tree_.threshold[0], rel=1e-6)


def test_grown_tree_fits_distinct_training_points():
    X, y = _data(120, 4, 21)
    t = tree.fit(X, y, max_depth=64, min_split=2, min_leaf=1)
    assert np.array_equal(tree.predict(t, X), y)
    # every child follows its parent (the library relies on it)
    for k, f in enumerate(t["feature"]):
        if f >= 0:
            assert t["left"][k] > k and t["right"][k] > k


def test_match_ratios_by_hand():
    pred = [8, 10, 0, 4, 12]
    truth = [8, 2, 0, 1, 14]
    exact, partial = tree.match_ratios(pred, truth)
    assert exact == pytest.approx(2 / 5)      # 8 == 8, 0 == 0
    assert partial == pytest.approx(4 / 5)    # 4 vs 1 share no class


def test_committed_tree_reproduces_its_training_record():
    d = json.load(open(tree.TREE))
    recs = learn.read_labels(os.path.join(os.path.dirname(tree.TREE), d["meta"]["labels"]))
    X = np.array([r["features"] for r in recs])
    y = np.array([r[d["meta"]["key"]] for r in recs])
    t = tree.load()
    assert tree.match_ratios(tree.predict(t, X), y)[0] == pytest.approx(d["meta"]["train_exact_match"])
    assert tree.fit(X, y, max_depth=d["meta"]["max_depth"]) == t


def test_library_rejects_malformed_trees():
    ok = {"feature": [0, -1, -1], "threshold": [0.5, 0.0, 0.0], "left": [1, -1, -1],
          "right": [2, -1, -1], "value": [0, 8, 12]}
    pkg.tree_load(ok)
    for key, bad in (("left", [0, -1, -1]), ("feature", [16, -1, -1]), ("value", [0, 16, 12]),
                     ("threshold", [float("nan"), 0.0, 0.0])):
        t = dict(ok, **{key: bad})
        with pytest.raises(pkg.CsrError):
            pkg.tree_load(t)
    pkg.tree_unload()

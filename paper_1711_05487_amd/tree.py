"""The paper's feature-guided classifier (Sec. III-D): a CART decision tree
over the 16 matrix features that predicts the bottleneck classes the
profile-guided classifier (Sec. III-C, Fig. 4) would assign, as a multilabel
problem (one output per class MB, ML, IMB, CMP; the empty set is the paper's
"dummy class" of matrices not worth optimizing). The predicted classes map to
remedies through Table II, as on the profile path.

Training runs here on the host (it is offline and small); the library walks
the exported tree after csr_inspect (CSR_SEL_TREE). Accuracy is reported as
the paper does, by the Exact Match Ratio (predicted set equal to the label
set) and the Partial Match Ratio (at least one class in common), under
k-fold cross-validation.

    python -m paper_1711_05487_amd.tree train --labels bounds.jsonl --key classes

The labels are the class masks the profile rule assigned when the records
were taken: `classes` of the bounds records (`learn bounds`, the rule with
the library's thresholds) or `profile_classes` of the timing labels
(`learn label`).
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_CLASSES = 4  # MB, ML, IMB, CMP: bits 0..3 of the class mask
TREE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "tree_mi355x.json")


def masks_to_bits(masks) -> np.ndarray:
    m = np.asarray(masks, dtype=np.int64)
    return ((m[:, None] >> np.arange(N_CLASSES)) & 1).astype(np.int64)


def bits_to_masks(bits) -> np.ndarray:
    return (np.asarray(bits, dtype=np.int64) << np.arange(N_CLASSES)).sum(axis=1)


def gini(Y: np.ndarray) -> float:
    """Mean over the outputs of the Gini impurity 1 - p0^2 - p1^2 of the
    0/1 labels Y (rows = samples)."""
    if len(Y) == 0:
        return 0.0
    p = Y.mean(axis=0)
    return float(np.mean(1.0 - p * p - (1.0 - p) * (1.0 - p)))


def best_split(X: np.ndarray, Y: np.ndarray, min_leaf: int):
    """The split (feature, threshold) of largest impurity decrease
    n*G(all) - nL*G(left) - nR*G(right), left = {x_f <= threshold},
    thresholds at midpoints of consecutive distinct values; ties go to the
    lower feature, then the lower threshold. None when no split leaves at
    least `min_leaf` samples on each side or none decreases the impurity."""
    n = len(X)
    parent = n * gini(Y)
    best = None
    if n < 2 * min_leaf:
        return None
    k = np.arange(n - 1)
    nl = (k + 1).astype(np.float64)[:, None]
    nr = (n - k - 1).astype(np.float64)[:, None]
    ok = (k >= min_leaf - 1) & (k < n - min_leaf)
    for f in range(X.shape[1]):
        order = np.argsort(X[:, f], kind="stable")
        xs, ys = X[order, f], Y[order].astype(np.float64)
        cum = np.cumsum(ys, axis=0)[:-1]      # positives among the first k+1 samples
        tot = ys.sum(axis=0)
        pl, pr = cum / nl, (tot - cum) / nr
        gl = np.mean(1.0 - pl * pl - (1.0 - pl) ** 2, axis=1)
        gr = np.mean(1.0 - pr * pr - (1.0 - pr) ** 2, axis=1)
        dec = parent - nl[:, 0] * gl - nr[:, 0] * gr
        valid = ok & (xs[:-1] != xs[1:]) & (dec > 1e-12)
        if not valid.any():
            continue
        d = np.where(valid, dec, -np.inf)
        j = int(np.argmax(d))                 # first (lowest threshold) of the best
        if best is None or d[j] > best[0] + 1e-12:
            best = (float(d[j]), f, 0.5 * (xs[j] + xs[j + 1]))
    return None if best is None else (best[1], best[2])


def fit(X, masks, max_depth: int = 10, min_split: int = 4, min_leaf: int = 2) -> dict:
    """CART (Breiman et al. 1984) for the multilabel class sets. Returns the
    tree as flat arrays: feature (-1 at leaves), threshold, left, right, and
    value (the class mask of a leaf: per class, the majority of its samples,
    a tie reading 0)."""
    X = np.asarray(X, dtype=np.float64)
    Y = masks_to_bits(masks)
    nodes = {"feature": [], "threshold": [], "left": [], "right": [], "value": []}

    def leaf_value(idx):
        pos = Y[idx].sum(axis=0)
        return int(bits_to_masks((2 * pos > len(idx)).astype(np.int64)[None, :])[0])

    def grow(idx, depth):
        k = len(nodes["feature"])
        for a in nodes:
            nodes[a].append(0)
        nodes["feature"][k], nodes["left"][k], nodes["right"][k] = -1, -1, -1
        nodes["threshold"][k] = 0.0
        nodes["value"][k] = leaf_value(idx)
        if depth >= max_depth or len(idx) < min_split or gini(Y[idx]) == 0.0:
            return k
        sp = best_split(X[idx], Y[idx], min_leaf)
        if sp is None:
            return k
        f, thr = sp
        go_left = X[idx, f] <= thr
        nodes["feature"][k], nodes["threshold"][k] = int(f), float(thr)
        nodes["left"][k] = grow(idx[go_left], depth + 1)
        nodes["right"][k] = grow(idx[~go_left], depth + 1)
        return k

    grow(np.arange(len(X)), 0)
    return nodes


def predict(tree: dict, X) -> np.ndarray:
    X = np.asarray(X, dtype=np.float64)
    out = np.empty(len(X), dtype=np.int64)
    for i, x in enumerate(X):
        k = 0
        while tree["feature"][k] >= 0:
            k = tree["left"][k] if x[tree["feature"][k]] <= tree["threshold"][k] else tree["right"][k]
        out[i] = tree["value"][k]
    return out


def match_ratios(pred, truth):
    """(Exact Match Ratio, Partial Match Ratio) of Sec. IV-B: the share of
    samples whose predicted set equals the label set, and the share whose
    prediction has at least one class in common with it (two empty sets
    count as a match)."""
    pred, truth = np.asarray(pred), np.asarray(truth)
    exact = pred == truth
    partial = ((pred & truth) != 0) | exact
    return float(exact.mean()), float(partial.mean())


def cross_validate(X, masks, folds: int = 10, **kw):
    """k-fold cross-validation (fold of sample i = i mod k): mean Exact and
    Partial Match Ratios over the folds."""
    X = np.asarray(X, dtype=np.float64)
    masks = np.asarray(masks, dtype=np.int64)
    ex, pa = [], []
    for k in range(folds):
        te = np.arange(len(X)) % folds == k
        t = fit(X[~te], masks[~te], **kw)
        e, p = match_ratios(predict(t, X[te]), masks[te])
        ex.append(e)
        pa.append(p)
    return float(np.mean(ex)), float(np.mean(pa))


def save(tree: dict, path: str, meta: dict | None = None):
    with open(path, "w") as f:
        json.dump({"format": "csr-cart-1", "n_features": 16, "classes": ["MB", "ML", "IMB", "CMP"],
                   **tree, "meta": meta or {}}, f)


def load(path: str = TREE) -> dict:
    with open(path) as f:
        d = json.load(f)
    return {k: d[k] for k in ("feature", "threshold", "left", "right", "value")}


def install(path: str = TREE):
    """Load the tree into the library (csr_tree_load) for CSR_SEL_TREE."""
    import paper_1711_05487_amd as pkg
    pkg.tree_load(load(path))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--labels", required=True)
    t.add_argument("--out", default=TREE)
    t.add_argument("--key", default="classes", help="record field holding the class mask")
    t.add_argument("--max-depth", type=int, default=0,
                   help="0: the depth of best cross-validated exact match, 2 .. 10")
    t.add_argument("--folds", type=int, default=10)
    a = ap.parse_args()
    from paper_1711_05487_amd import learn
    recs = learn.read_labels(a.labels)
    X = np.array([r["features"] for r in recs])
    y = np.array([r[a.key] for r in recs], dtype=np.int64)
    depth, by_depth = a.max_depth, {}
    if depth <= 0:
        for d in range(2, 11):
            by_depth[d] = cross_validate(X, y, folds=a.folds, max_depth=d)
        depth = max(by_depth, key=lambda d: (by_depth[d][0], -d))
    exact, partial = by_depth.get(depth) or cross_validate(X, y, folds=a.folds, max_depth=depth)
    tree = fit(X, y, max_depth=depth)
    train_exact, train_partial = match_ratios(predict(tree, X), y)
    meta = {"samples": len(recs), "labels": os.path.basename(a.labels), "key": a.key,
            "folds": a.folds, "max_depth": depth,
            "cv_exact_match_by_depth": {str(d): v[0] for d, v in by_depth.items()},
            "cv_exact_match": exact, "cv_partial_match": partial,
            "train_exact_match": train_exact, "train_partial_match": train_partial,
            "nodes": len(tree["feature"]),
            "label_masks": {str(m): int((y == m).sum()) for m in sorted(set(y.tolist()))}}
    save(tree, a.out, meta)
    print(json.dumps(meta, indent=1))


if __name__ == "__main__":
    main()

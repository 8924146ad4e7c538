"""Training driver of the learned selector (replaces the decision tree of the
feature-guided classifier, Sec. III-D).

  label  time all 16 catalogue variants of every matrix of the seeded suite on
         the current GPU (the fastest is the label, ties to the lower id) and
         record the features, all times and the profile-guided classes as
         JSON lines (append-only, resumable by matrix index);
  train  fit the MLP 16-64-64-16 on those labels with the library's own
         forward/backward/Adam kernels (csr_mlp_train) and save the weights.

    python -m paper_1711_05487_amd.learn label --start 0 --count 2000 --out labels.jsonl
    python -m paper_1711_05487_amd.learn train --labels labels.jsonl --out weights.json

The suite is synthetic (seeded generators), standing in for the University
of Florida matrices the paper trains on.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

K = 16
SIZES = [16, 64, 64, K]
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "mlp16_mi355x.json")


# ---------------------------------------------------------------------------
# Labeling
# ---------------------------------------------------------------------------

def _gen_to_file(args):
    """Worker (CPU only): generate suite matrix `index` into an .npz file."""
    index, base_seed, n_min, n_max, nnz_cap, tmpdir = args
    import synth
    name, (n, m, rp, col, val) = synth.suite_matrix(index, base_seed=base_seed, n_min=n_min,
                                                   n_max=n_max, nnz_cap=nnz_cap)
    path = os.path.join(tmpdir, f"m{index}.npy")
    with open(path, "wb") as f:
        np.save(f, np.array([n, m, len(col)], dtype=np.int64))
        np.save(f, rp)
        np.save(f, col)
        np.save(f, val)
    return index, name, path


def _load(path):
    with open(path, "rb") as f:
        n, m, nnz = np.load(f)
        rp, col, val = np.load(f), np.load(f), np.load(f)
    os.remove(path)
    return int(n), int(m), rp, col, val


def time_variants(A, xd, yd, calls=10, runs=3):
    """Time every catalogue variant (default parameters) with events on the
    current stream. Returns ms per call for variant ids 0..15."""
    import torch
    out = []
    s = torch.cuda.current_stream()
    for v in catalogue():
        A.select("forced", forced_opts=v)
        A.spmv(xd, yd)
        ts = []
        for _ in range(runs):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(calls):
                A.spmv(xd, yd)
            e1.record(s)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) / calls)
        out.append(float(np.mean(ts)))
    return out


def catalogue():
    """Optimization sets of the 16 variants (ids as in the library)."""
    o = [1, 2, 4, 8, 16]
    sets = [0] + o
    for a in range(5):
        for b in range(a + 1, 5):
            sets.append(o[a] | o[b])
    return sets


def label(start, count, out, base_seed=501, n_min=1e4, n_max=4e6, nnz_cap=1 << 25, workers=8,
          calls=10, runs=3):
    import multiprocessing as mp
    import torch
    import paper_1711_05487_amd as pkg

    done = set()
    if os.path.exists(out):
        with open(out) as f:
            for line in f:
                try:
                    done.add(json.loads(line)["index"])
                except Exception:
                    pass
    todo = [i for i in range(start, start + count) if i not in done]
    print(f"[label] {len(todo)} matrices to label ({len(done)} already in {out})", flush=True)
    if not todo:
        return
    gpu = torch.cuda.get_device_name(0)
    tmpdir = tempfile.mkdtemp(prefix="csr_suite_", dir="/dev/shm" if os.path.isdir("/dev/shm") else None)
    ctx = mp.get_context("spawn")
    t0 = time.time()
    with ctx.Pool(workers) as pool, open(out, "a") as fo:
        jobs = [(i, base_seed, n_min, n_max, nnz_cap, tmpdir) for i in todo]
        for k, (index, name, path) in enumerate(pool.imap(_gen_to_file, jobs)):
            n, m, rp, col, val = _load(path)
            A = pkg.CsrMatrix(rp, col, val, n_cols=m)
            f, isum, sorted_flag = A.inspect()
            xd = torch.ones(m, dtype=torch.float64, device="cuda")
            yd = torch.empty(n, dtype=torch.float64, device="cuda")
            times = time_variants(A, xd, yd, calls, runs)
            prof = A.select("profile", timing_calls=calls)
            best = int(np.argmin(times))
            rec = {"index": index, "seed": base_seed + index, "name": name, "n": n, "nnz": len(col),
                   "features": [float(v) for v in f], "isum": [int(v) for v in isum],
                   "sorted": int(sorted_flag), "times_ms": times, "label": best,
                   "profile_classes": prof["classes"], "profile_opts": prof["opts"],
                   "profile_variant": prof["variant_id"], "profile_select_ms": prof["t_select_ms"],
                   "gpu": gpu}
            A.spmv(xd, yd)
            torch.cuda.synchronize()
            rec["profile_ms"] = _time_current(A, xd, yd, calls, runs)
            fo.write(json.dumps(rec) + "\n")
            fo.flush()
            A.close()
            print(f"[label] {k + 1}/{len(todo)} idx={index} {name} n={n} nnz={len(col)} "
                  f"best={best} t_best={min(times):.4f}ms t_plain={times[0]:.4f}ms "
                  f"({time.time() - t0:.0f}s)", flush=True)
    os.rmdir(tmpdir)


def _remedies_of(pkg, cls, has_long, remedy_map):
    # classes -> remedies under the library's map: the bounds are chosen so
    # that the library's rule returns exactly `cls` (each class's test made
    # to hold or fail on its own), which keeps the map in one place (the
    # library)
    p = {"csr": 1.0, "mb": 1.0, "ml": 1.0, "imb": 1.0, "cmp": 1.0, "peak": 1.0}
    cfg = pkg.default_config()
    cfg.t_ml, cfg.t_imb, cfg.t_mb = 1.5, 1.5, 0.5
    cfg.remedy_map = remedy_map
    if cls & 4:
        p["imb"] = 2.0
    if cls & 2:
        p["ml"] = 2.0
    if cls & 1:      # P_CSR >= t_mb P_MB and P_MB < P_CMP < P_peak
        p.update(mb=1.5, cmp=1.7, peak=2.0)
    elif cls & 8:    # P_CMP < P_MB
        p.update(mb=1.5, cmp=1.2, peak=2.0)
    else:            # neither: P_CMP == P_MB (not below, not strictly between)
        p.update(mb=1.5, cmp=1.5, peak=2.0)
    if (cls & 1) and (cls & 8):
        return None  # MB and CMP exclude each other under the rule
    got, opts = pkg.classify([p[k] for k in ("csr", "mb", "ml", "imb", "cmp", "peak")],
                             has_long, config=cfg)
    assert got == cls, (cls, got)
    return opts


def profile_label(start, count, out, base_seed=501, n_min=1e4, n_max=4e6, nnz_cap=1 << 25,
                  workers=8, calls=10, runs=3):
    """For the threshold grid search of the profile-guided classifier
    (Sec. III-C): per matrix, the bounds of Sec. III-B as PROFILE measures
    them, the time of every optimization set the rule can pick (one per
    class mask, default parameters) and, for the regret judge, the 16
    catalogue variants timed in the same session. JSON lines, resumable."""
    import multiprocessing as mp
    import torch
    import paper_1711_05487_amd as pkg

    done = set()
    if os.path.exists(out):
        with open(out) as f:
            for line in f:
                try:
                    done.add(json.loads(line)["index"])
                except Exception:
                    pass
    todo = [i for i in range(start, start + count) if i not in done]
    print(f"[bounds] {len(todo)} matrices ({len(done)} already in {out})", flush=True)
    if not todo:
        return
    tmpdir = tempfile.mkdtemp(prefix="csr_bounds_", dir="/dev/shm" if os.path.isdir("/dev/shm") else None)
    ctx = mp.get_context("spawn")
    t0 = time.time()
    cfg_tau = pkg.default_config()
    with ctx.Pool(workers) as pool, open(out, "a") as fo:
        jobs = [(i, base_seed, n_min, n_max, nnz_cap, tmpdir) for i in todo]
        for k, (index, name, path) in enumerate(pool.imap(_gen_to_file, jobs)):
            n, m, rp, col, val = _load(path)
            A = pkg.CsrMatrix(rp, col, val, n_cols=m)
            f, isum, sorted_flag = A.inspect()
            tau = max(cfg_tau.long_row_factor * f[3], cfg_tau.long_row_floor)
            has_long = bool(f[2] > tau)
            prof = A.select("profile", autotune=0, timing_calls=calls)
            xd = torch.ones(m, dtype=torch.float64, device="cuda")
            yd = torch.empty(n, dtype=torch.float64, device="cuda")
            set_times = {}
            reach = {_remedies_of(pkg, c, has_long, mp_) for c in range(16) for mp_ in (0, 1)}
            for opts in sorted({canonical_opts(o) for o in reach if o is not None}):
                A.select("forced", forced_opts=opts)
                A.spmv(xd, yd)
                set_times[str(opts)] = _time_current(A, xd, yd, calls, runs)
            cat = time_variants(A, xd, yd, calls, runs)
            rec = {"index": index, "seed": base_seed + index, "name": name, "n": n,
                   "nnz": len(col), "features": [float(v) for v in f], "has_long": has_long,
                   "bounds": [prof[k] for k in ("p_csr", "p_mb", "p_ml", "p_imb", "p_cmp",
                                                "p_peak")],
                   "b_max": prof["b_max"], "classes": prof["classes"], "opts": prof["opts"],
                   "set_times_ms": set_times, "catalogue_ms": cat}
            fo.write(json.dumps(rec) + "\n")
            fo.flush()
            A.close()
            print(f"[bounds] {k + 1}/{len(todo)} idx={index} {name} n={n} nnz={len(col)} "
                  f"classes={prof['classes']} ({time.time() - t0:.0f}s)", flush=True)
    os.rmdir(tmpdir)


def canonical_opts(opts):
    """The optimization set the library actually realizes: the merge path
    takes precedence over long-row decomposition, so MERGE|DECOMP runs the
    plan of MERGE."""
    return opts & ~4 if opts & 8 else opts


def set_time(rec, opts):
    """Time of an optimization set in a bounds record: from the sets timed
    for the rule, else from the catalogue timed in the same session."""
    o = canonical_opts(opts)
    st = rec["set_times_ms"]
    if str(o) in st:
        return st[str(o)]
    return rec["catalogue_ms"][catalogue().index(o)]


# the paper's thresholds, tuned on its KNC platform (Sec. IV-B)
PAPER_THRESHOLDS = (1.25, 1.24, 0.8)


def default_thresholds():
    import paper_1711_05487_amd as pkg
    d = pkg.default_config()
    return (d.t_ml, d.t_imb, d.t_mb)


def tune_thresholds(recs, remedy_map=1, grid_ml=None, grid_imb=None, grid_mb=None,
                    defaults=None):
    """Grid search of T_ML, T_IMB and T_MB (Sec. III-C: the thresholds are the
    classifier's hyperparameters, tuned by exhaustive grid search for the
    highest average performance gain of the chosen optimizations): for every
    setting, every record's classes under the library's rule, the time of
    the set they map to under `remedy_map`, and the mean of t_plain / t_set.
    Returns (best (t_ml, t_imb, t_mb), its mean gain, the mean gain of
    `defaults`, the library's defaults when None)."""
    import paper_1711_05487_amd as pkg
    grid_ml = np.round(np.arange(1.0, 3.001, 0.05), 4) if grid_ml is None else grid_ml
    grid_imb = np.round(np.arange(1.0, 3.001, 0.05), 4) if grid_imb is None else grid_imb
    grid_mb = np.round(np.arange(0.5, 1.001, 0.05), 4) if grid_mb is None else grid_mb

    def gain(t_ml, t_imb, t_mb):
        cfg = pkg.default_config()
        cfg.t_ml, cfg.t_imb, cfg.t_mb = float(t_ml), float(t_imb), float(t_mb)
        cfg.remedy_map = remedy_map
        g = []
        for r in recs:
            _, opts = pkg.classify(r["bounds"], r["has_long"], config=cfg)
            g.append(r["set_times_ms"]["0"] / set_time(r, opts))
        return float(np.mean(g))

    best, best_g = None, -1.0
    for a in grid_ml:
        for b in grid_imb:
            for c in grid_mb:
                v = gain(a, b, c)
                if v > best_g + 1e-12:
                    best, best_g = (float(a), float(b), float(c)), v
    d = default_thresholds() if defaults is None else defaults
    return best, best_g, gain(*d)


def profile_regret(recs, thresholds, remedy_map=1):
    """Per record t_selected / t_best with the profile rule at the given
    thresholds (default parameters), t_best the fastest of everything timed
    for that matrix in the same session (16 catalogue variants and the sets
    the rule can pick). Returns (geomean, p90, geomean speedup over plain)."""
    import paper_1711_05487_amd as pkg
    cfg = pkg.default_config()
    cfg.t_ml, cfg.t_imb, cfg.t_mb = thresholds
    cfg.remedy_map = remedy_map
    ratio, speed = [], []
    for r in recs:
        _, opts = pkg.classify(r["bounds"], r["has_long"], config=cfg)
        t = set_time(r, opts)
        best = min(min(r["catalogue_ms"]), min(r["set_times_ms"].values()))
        ratio.append(t / best)
        speed.append(r["set_times_ms"]["0"] / t)
    gm = lambda a: float(np.exp(np.mean(np.log(a))))
    return gm(ratio), float(np.percentile(ratio, 90)), gm(speed)


def _time_current(A, xd, yd, calls, runs):
    import torch
    s = torch.cuda.current_stream()
    ts = []
    for _ in range(runs):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(calls):
            A.spmv(xd, yd)
        e1.record(s)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) / calls)
    return float(np.mean(ts))


# ---------------------------------------------------------------------------
# Training
# ---------------------------------------------------------------------------

def read_labels(path):
    recs = []
    with open(path) as f:
        for line in f:
            recs.append(json.loads(line))
    recs.sort(key=lambda r: r["index"])
    return recs


def split(recs, seed=703, test_frac=0.2):
    """80/20 split by matrix seed (a hash of the seed, not the position)."""
    import synth
    tr, te = [], []
    for r in recs:
        u = float(synth.u01(seed, 0, np.array([r["seed"]], dtype=np.uint64))[0])
        (te if u <= test_frac else tr).append(r)
    return tr, te


def normalization(recs):
    F = np.log2(1.0 + np.array([r["features"] for r in recs], dtype=np.float64))
    mu = F.mean(axis=0)
    sd = F.std(axis=0)
    sd[sd < 1e-6] = 1.0
    return mu, sd


def train(recs, epochs=200, batch=64, lr=1e-3, init_seed=701, shuffle_seed=702):
    """Fit the MLP on GPU with the library's kernels. Returns (params, mu,
    sigma, losses)."""
    import torch
    import paper_1711_05487_amd as pkg
    import synth
    mu, sd = normalization(recs)
    F = torch.tensor(np.array([r["features"] for r in recs], dtype=np.float64), device="cuda")
    X = pkg.mlp_normalize(F, torch.tensor(mu, device="cuda"), torch.tensor(sd, device="cuda"))
    y = torch.tensor([r["label"] for r in recs], dtype=torch.int32, device="cuda")
    params = torch.tensor(np.concatenate([p.ravel() for p in synth.mlp_init_weights(SIZES, init_seed)]),
                          dtype=torch.float32, device="cuda")
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    n = len(recs)
    B = min(batch, n)
    steps_per_epoch = n // B
    order = []
    for e in range(epochs):
        perm = synth.permutation(n, shuffle_seed, stream=e)
        order.append(perm[:steps_per_epoch * B])
    order = torch.tensor(np.concatenate(order), dtype=torch.int32, device="cuda")
    losses = pkg.mlp_train(params, m, v, K, X, y, order, B, t0=0, lr=lr)
    return params.cpu().numpy(), mu, sd, losses.cpu().numpy()


def predict(params, mu, sd, feats):
    import torch
    import paper_1711_05487_amd as pkg
    F = torch.tensor(np.asarray(feats, dtype=np.float64), device="cuda")
    X = pkg.mlp_normalize(F, torch.tensor(mu, device="cuda"), torch.tensor(sd, device="cuda"))
    P = torch.tensor(params, device="cuda")
    out = []
    for b in range(0, X.shape[0], 64):
        logits = pkg.mlp_forward(P, K, X[b:b + 64].contiguous())
        out.append(torch.argmax(logits, dim=1).cpu().numpy())
    return np.concatenate(out) if out else np.zeros(0, dtype=np.int64)


def evaluate(recs, pred):
    """Per matrix: selected / best time (regret + 1), also for the baseline
    and for the profile-guided choice recorded at labeling time."""
    t = np.array([r["times_ms"] for r in recs])
    best = t.min(axis=1)
    sel = t[np.arange(len(recs)), pred]
    prof = np.array([r.get("profile_ms", np.nan) for r in recs])
    gm = lambda a: float(np.exp(np.mean(np.log(a))))
    return {
        "n": len(recs),
        "geomean_sel_over_best": gm(sel / best),
        "p90_sel_over_best": float(np.percentile(sel / best, 90)),
        "geomean_plain_over_best": gm(t[:, 0] / best),
        "geomean_profile_over_best": gm(prof / best) if np.isfinite(prof).all() else None,
        "geomean_speedup_vs_plain": gm(t[:, 0] / sel),
        "accuracy": float(np.mean(pred == np.argmin(t, axis=1))),
    }


class WeightsError(ValueError):
    """A weights file that is malformed or fails its checksum."""


def weights_digest(params, mu, sd) -> str:
    """SHA-256 over the model's bytes: FP32 parameters, then FP64 mu and sigma."""
    import hashlib
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(params, dtype="<f4").tobytes())
    h.update(np.ascontiguousarray(mu, dtype="<f8").tobytes())
    h.update(np.ascontiguousarray(sd, dtype="<f8").tobytes())
    return h.hexdigest()


def save_weights(path, params, mu, sd, meta):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    params = np.asarray(params, dtype=np.float32)
    with open(path, "w") as f:
        json.dump({"K": K, "sizes": SIZES, "params": [float(v) for v in params],
                   "mu": [float(v) for v in mu], "sigma": [float(v) for v in sd],
                   "sha256": weights_digest(params, mu, sd), "meta": meta}, f)


def load_weights(path=WEIGHTS):
    """(params, mu, sigma, meta) of a saved model; WeightsError when the file
    is malformed, has the wrong shapes or does not match its checksum."""
    try:
        with open(path) as f:
            d = json.load(f)
        params = np.array(d["params"], dtype=np.float32)
        mu, sd = np.array(d["mu"], dtype=np.float64), np.array(d["sigma"], dtype=np.float64)
        digest = d["sha256"]
    except (OSError, ValueError, KeyError, TypeError) as e:
        raise WeightsError(f"{path}: unreadable weights ({e})") from None
    n = sum(SIZES[i + 1] * SIZES[i] + SIZES[i + 1] for i in range(len(SIZES) - 1))
    if params.shape != (n,) or mu.shape != (16,) or sd.shape != (16,):
        raise WeightsError(f"{path}: wrong shapes")
    if weights_digest(params, mu, sd) != digest:
        raise WeightsError(f"{path}: checksum mismatch")
    return params, mu, sd, d.get("meta", {})


def install(path=WEIGHTS) -> bool:
    """Load the saved model into the library for select('learned'). A
    corrupted or unreadable file installs nothing (any model loaded before
    is removed, so learned selection falls back to the profile-guided one)
    and returns False."""
    import paper_1711_05487_amd as pkg
    try:
        params, mu, sd, _ = load_weights(path)
    except WeightsError as e:
        print(f"[learn] not installing the selector model: {e}", file=sys.stderr)
        pkg.mlp_unload()
        return False
    pkg.mlp_load(params, K, mu, sd)
    return True


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("label")
    a.add_argument("--start", type=int, default=0)
    a.add_argument("--count", type=int, default=2000)
    a.add_argument("--out", required=True)
    a.add_argument("--workers", type=int, default=8)
    a.add_argument("--n-max", type=float, default=4e6)
    c = sub.add_parser("bounds")
    c.add_argument("--start", type=int, default=0)
    c.add_argument("--count", type=int, default=400)
    c.add_argument("--out", required=True)
    c.add_argument("--workers", type=int, default=8)
    c.add_argument("--n-max", type=float, default=4e6)
    c.add_argument("--calls", type=int, default=32)
    t = sub.add_parser("tune")
    t.add_argument("--bounds", required=True)
    b = sub.add_parser("train")
    b.add_argument("--labels", required=True)
    b.add_argument("--out", default=WEIGHTS)
    b.add_argument("--epochs", type=int, default=200)
    args = ap.parse_args()
    if args.cmd == "label":
        label(args.start, args.count, args.out, workers=args.workers, n_max=args.n_max)
    elif args.cmd == "bounds":
        profile_label(args.start, args.count, args.out, workers=args.workers, n_max=args.n_max,
                      calls=args.calls)
    elif args.cmd == "tune":
        recs = read_labels(args.bounds)
        tr, te = split(recs)
        out = {"n_train": len(tr), "n_test": len(te), "default": default_thresholds(),
               "paper": PAPER_THRESHOLDS}
        for mp_ in (0, 1):
            best, g_best, g_paper = tune_thresholds(tr, mp_, defaults=PAPER_THRESHOLDS)
            out[f"map{mp_}"] = {
                "best": best, "train_gain_best": g_best, "train_gain_paper": g_paper,
                "test_paper": profile_regret(te, PAPER_THRESHOLDS, mp_),
                "test_best": profile_regret(te, best, mp_)}
        print(json.dumps(out, indent=1), flush=True)
    else:
        recs = read_labels(args.labels)
        tr, te = split(recs)
        params, mu, sd, losses = train(tr, epochs=args.epochs)
        ev_tr = evaluate(tr, predict(params, mu, sd, [r["features"] for r in tr]))
        ev_te = evaluate(te, predict(params, mu, sd, [r["features"] for r in te]))
        meta = {"train": ev_tr, "test": ev_te, "final_loss": float(losses[-1]),
                "epochs": args.epochs, "n_train": len(tr), "n_test": len(te),
                "gpu": recs[0].get("gpu") if recs else None}
        save_weights(args.out, params, mu, sd, meta)
        print(json.dumps(meta, indent=1), flush=True)


if __name__ == "__main__":
    main()

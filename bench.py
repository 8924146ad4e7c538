"""Benchmark: SpMV effective HBM GB/s of the selected variant vs plain CSR.

One step = one y = A x with the plan chosen by the selector (default: the
learned selector with the committed model), on the 27-point stencil over a
128^3 grid (N = 2,097,152, NNZ = 55,742,968, FP64 values, int32 indices),
inputs resident in HBM. The selector runs once before the timed region (the
inspector/executor split of the method); its cost is reported beside the
rate, with the solver-iteration count that amortizes it (Sec. IV-D, Eq. (2)).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--select learned|profile|exhaustive|plain]
    python bench.py --suite     # every configuration, one JSON line per case

Prints one JSON line (the suite: one per case). The product path is
checked on the GPU against the plain row-split kernel (FP64: within
2e-12 (|A||x|)_i, the scale from a second SpMV with |A| and |x|); the
oracle is only timed, as the CPU baseline, and the parity tests compare
every kernel with it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "SpMV effective HBM GB/s (% of peak) + speedup of selected variant vs plain CSR"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def harmonic_runs(A, x, y, runs, calls):
    """Sec. IV-A protocol: rate of each run = work / time over `calls` warm
    back-to-back SpMVs; summary = harmonic mean over runs. Returns ms/call."""
    import torch
    s = torch.cuda.current_stream()
    A.spmv(x, y)
    t = []
    for _ in range(runs):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(calls):
            A.spmv(x, y)
        e1.record(s)
        e1.synchronize()
        t.append(e0.elapsed_time(e1) / calls)
    return float(np.mean(t))  # 1 / harmonic mean of rates = arithmetic mean of times


def n_iters_min(t_pre_ms, t_plain_ms, t_sel_ms):
    """Solver iterations that amortize selection and preprocessing
    (Sec. IV-D, Eq. (2)); None when the selected variant is not faster."""
    return t_pre_ms / (t_plain_ms - t_sel_ms) if t_sel_ms < t_plain_ms else None


class GpuCheck:
    """The product path checked on the GPU: the plain row-split result and
    the per-row scale (|A||x|)_i from a plain SpMV of |A| with |x|."""

    def __init__(self, pkg, rp, col, val, x, n_cols):
        import torch
        self.x = torch.from_numpy(x).cuda()
        P = pkg.CsrMatrix(rp, col, val, n_cols=n_cols)
        self.y_plain = P.spmv(self.x)
        Q = pkg.CsrMatrix(rp, col, np.abs(val), n_cols=n_cols)
        self.absax = Q.spmv(self.x.abs())
        torch.cuda.synchronize()
        P.close()
        Q.close()

    def f64_ok(self, y):
        import torch
        return bool(torch.all((y - self.y_plain).abs() <= 2e-12 * self.absax).item())

    def rel_errors(self, y):
        """max and 99th percentile over rows of |y - y_f64| / (|A||x|)_i."""
        import torch
        ab = self.absax
        m = ab > 0
        rel = ((y.double() - self.y_plain).abs()[m] / ab[m]).cpu().numpy()
        if rel.size == 0:
            return 0.0, 0.0
        return float(rel.max()), float(np.percentile(rel, 99))


# the sources of the merge-path kernel and of the encodings it reads: a change
# to any of them invalidates counter data taken before it
KERNEL_SOURCES = ("paper_1711_05487_amd/csrc/k_merge.hip", "paper_1711_05487_amd/csrc/merge_kernel.h",
                  "paper_1711_05487_amd/csrc/merge_tile.h", "paper_1711_05487_amd/csrc/device.h",
                  "paper_1711_05487_amd/csrc/kdefs.h", "paper_1711_05487_amd/csrc/internal.h",
                  "paper_1711_05487_amd/csrc/k_prep.hip", "include/csrspmv.h")


def code_text(src: str) -> str:
    """C/C++ source with comments removed and whitespace runs collapsed, so
    that edits to comments alone leave the hash unchanged (string literals
    in these sources hold no comment markers)."""
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def kernel_source_sha(texts=None):
    """Hash of the code (not the comments) of KERNEL_SOURCES, or of the given
    texts in that order."""
    h = hashlib.sha256()
    if texts is None:
        texts = [open(os.path.join(ROOT, f)).read() for f in KERNEL_SOURCES]
    for t in texts:
        h.update(code_text(t).encode())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel, workload, launches_bytes):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel sources; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        rec = d.get(kernel)
        if not rec or rec.get("workload") != workload or rec.get("src_sha") != kernel_source_sha():
            return None
        return float(rec["hbm_bytes_per_launch"])
    except Exception:
        return None


def cpu_baseline(rp, col, val, x, bytes_per_call, budget_s=12.0, runs=5):
    """The oracle as it stands (single-threaded C, storage-order FP64), timed on
    the host: `runs` runs of whole-matrix calls of about budget_s / runs
    seconds each, summarized as the harmonic mean of the per-run rates
    (Sec. IV-A). Also returns the oracle's y for the parity check of the GPU
    result."""
    import oracle
    y = oracle.spmv(rp, col, val, x)  # warm; kept for the parity check
    rates, calls_total, el_total = [], 0, 0.0
    for _ in range(runs):
        t0 = time.perf_counter()
        calls = 0
        while True:
            oracle.spmv(rp, col, val, x)
            calls += 1
            el = time.perf_counter() - t0
            if el >= budget_s / runs or calls >= 1024:
                break
        rates.append(bytes_per_call * calls / el / 1e9)
        calls_total += calls
        el_total += el
    gbs = len(rates) / sum(1.0 / r for r in rates)
    rec = {"value": round(gbs, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
           "sample": f"{runs} runs, {calls_total} full SpMV calls of the same 27-point 128^3 FP64 "
                     f"matrix ({el_total:.1f} s, single thread), harmonic mean of the run rates"}
    return rec, y


def oracle_parity(y_gpu, y_oracle, rp, col, val, x):
    """The GPU result against the oracle's storage-order FP64 product from the
    CPU-baseline leg: both lie within gamma_n (|A||x|)_i of the exact product
    (n <= 27 here, gamma_n < 3e-15), so 1e-12 (|A||x|)_i bounds their gap."""
    import oracle
    ab = oracle.absax(rp, col, val, x)
    d = np.abs(np.asarray(y_gpu, dtype=np.float64) - y_oracle)
    nz = ab > 0
    ok = bool(np.all(d <= 1e-12 * ab)) and bool(np.all(d[~nz] == 0))
    rel = float(np.max(d[nz] / ab[nz])) if nz.any() else 0.0
    return {"ok": ok, "max_rel": rel, "bar": "1e-12 (|A||x|)_i per row, against the oracle"}


def cpu_multicore(rp, col, val, x, bytes_per_call, budget_s=4.0):
    """The OpenMP CSR baseline (Sec. IV-A: contiguous nnz-balanced row blocks,
    one per thread) on all host threads OpenMP is given: context beside the
    single-threaded oracle, never the target."""
    import cpu_omp
    sec, th = cpu_omp.time_spmv(rp, col, val, x, 4)
    calls = max(4, min(2048, int(budget_s / max(sec / 4, 1e-6))))
    sec, th = cpu_omp.time_spmv(rp, col, val, x, calls)
    return {"value": round(bytes_per_call * calls / sec / 1e9, 3), "unit": "GB/s", "threads": th,
            "kind": "openmp csr", "sample": f"{calls} full SpMV calls ({sec:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--select", default="learned",
                    help="learned (committed MLP), profile, exhaustive or plain")
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--suite", action="store_true",
                    help="measure every configuration (one JSON line per case)")
    ap.add_argument("--amortize", action="store_true",
                    help="amortization study (Sec. IV-D, Table V; one JSON line per case)")
    ap.add_argument("--amortize-matrices", type=int, default=40,
                    help="held-out suite matrices in the Table V study")
    ap.add_argument("--irregular", action="store_true",
                    help="run the irregular configurations' plans (R-MAT 22, uniform 2^20 x 16) "
                         "a few times each, for counter runs")
    ap.add_argument("--batch", action="store_true",
                    help="the 512-matrix batched launch alone (C5-batch; one JSON line)")
    ap.add_argument("--partitions", action="store_true",
                    help="partition-aware ML study: localized irregular stretches and a suite "
                         "sample under the profile rule with and without partitions")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU row sharding is a design, not a built path)", file=sys.stderr)
        sys.exit(2)

    if args.suite:
        return suite(args)
    if args.amortize:
        return amortize(args)
    if args.irregular:
        return irregular(args)
    if args.partitions:
        return partitions(args)
    if args.batch:
        return batch_only()

    import torch
    import paper_1711_05487_amd as pkg
    import synth
    from paper_1711_05487_amd import learn

    torch.cuda.set_device(0)
    n = args.grid
    log(f"generating 27-point stencil on {n}^3")
    N, M, rp, col, val = synth.stencil27(n)
    x = synth.vector(M, 203)
    nnz = len(col)
    workload = f"27-point stencil {n}^3 FP64 CSR (N={N:,}, NNZ={nnz:,})"
    t0 = time.perf_counter()
    A = pkg.CsrMatrix(rp, col, val)
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - t0) * 1e3
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty(N, dtype=torch.float64, device="cuda")

    log("triad (B_max probe)")
    triad = pkg.triad(1 << 30, 5) / 1e9

    log("plain row-split baseline")
    plain = A.select("plain")
    t_plain = harmonic_runs(A, xd, yd, 5, 128)
    plain_gbs = plain["format_bytes"] / (t_plain * 1e-3) / 1e9

    if args.select == "learned" and os.path.exists(learn.WEIGHTS):
        learn.install()
    # the first launch of each selection kernel in a process loads its code
    # object; that is a one-time process cost, not part of selecting for a
    # matrix, so the selector is run once on a small matrix first
    _, wm, wrp, wcol, wval = synth.laplacian2d(64)
    W = pkg.CsrMatrix(wrp, wcol, wval, n_cols=wm)
    W.select(args.select)
    W.close()
    log(f"selecting ({args.select})")
    info = A.select(args.select)

    # correctness gate on the selected plan (untimed): every row
    chk = GpuCheck(pkg, rp, col, val, x, M)
    A.spmv(xd, yd)
    torch.cuda.synchronize()
    ok = chk.f64_ok(yd)
    if not ok:
        log("PARITY FAILURE on the selected plan")

    log(f"timing {args.warmup} warmup + {args.steps} steps")
    s = torch.cuda.current_stream()
    for _ in range(args.warmup):
        A.spmv(xd, yd)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall0 = time.perf_counter()
    e0.record(s)
    for _ in range(args.steps):
        A.spmv(xd, yd)
    e1.record(s)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t_wall0) * 1e3
    ms = e0.elapsed_time(e1) / args.steps
    fmt_bytes = info["format_bytes"]
    gbs = fmt_bytes / (ms * 1e-3) / 1e9
    # the dominant kernel's mean duration from HIP events on its launch
    # stream: one event pair around 200 back-to-back calls of a one-kernel plan
    k_ms, call_ms, kernel = A.time_spmv(xd, yd, 200)
    achieved = fmt_bytes / (k_ms * 1e-3) / 1e9
    t_sel_proto = harmonic_runs(A, xd, yd, 5, 128)
    t_pre = info["t_select_ms"] + info["t_prep_ms"]

    opts = [name for bit, name in pkg.OPT_NAMES.items() if info["opts"] & bit]
    traffic = traffic_from_profiles(kernel, workload, fmt_bytes)
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": kernel, "kernel_ms": round(k_ms, 5),
            "algorithmic_bytes_per_launch": fmt_bytes}
    out = {
        "metric": METRIC,
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": workload,
            "selector": args.select,
            "selector_fallback": bool(info["fallback"]),
            "variant_opts": opts,
            "variant_id": info["variant_id"],
            "lanes_per_row": info["lanes_per_row"],
            "merge_items": info["merge_items"],
            "delta_bits": info["delta_bits"], "window_codes": bool(info["window_codes"]),
            "window_runs": info["window_codes"] == 2,
            "window_rank_bits": 9 if info["window_codes"] == 3 else 8 if info["window_codes"] else 0,
            "pct_of_hbm_peak": round(100 * gbs / HBM_PEAK_GBS, 2),
            "pct_of_triad": round(100 * gbs / triad, 2),
            "triad_gbs": round(triad, 1),
            "gflops": round(2 * nnz / (ms * 1e-3) / 1e9, 2),
            "plain_gbs": round(plain_gbs, 2),
            "plain_ms": round(t_plain, 5),
            "speedup_vs_plain": round(t_plain / ms, 4),
            "selected_ms_protocol": round(t_sel_proto, 5),
            "create_ms": round(create_ms, 2),
            "select_ms": round(info["t_select_ms"], 3),
            "prep_ms": round(info["t_prep_ms"], 3),
            "n_iters_min": (round(n_iters_min(t_pre, t_plain, ms), 1)
                            if ms < t_plain else None),
            "parity_ok": ok,
            "timed_wall_ms": round(wall_ms, 2),
        },
        "roofline": roof,
    }
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"], y_or = cpu_baseline(rp, col, val, x, plain["format_bytes"])
        A.spmv(xd, yd)
        torch.cuda.synchronize()
        par = oracle_parity(yd.cpu().numpy(), y_or, rp, col, val, x)
        out["config"]["parity_oracle"] = par
        ok = ok and par["ok"]
        out["config"]["parity_ok"] = ok
        log("cpu baseline (openmp)")
        out["cpu_multicore"] = cpu_multicore(rp, col, val, x, plain["format_bytes"])
    print(json.dumps(out), flush=True)
    A.close()
    if not ok:
        sys.exit(1)


# ---------------------------------------------------------------------------
# --suite: every configuration
# ---------------------------------------------------------------------------

def emit(rec):
    print(json.dumps(rec), flush=True)


def permuted(mat, seed=304):
    """Symmetric permutation P A P^T with a seeded Fisher-Yates permutation."""
    import synth
    n, m, rp, col, val = mat
    p = synth.permutation(n, seed)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    return synth.from_coo(p[rows], p[col.astype(np.int64)], val, n, m)


def time_plan(A, xd, yd, runs=5, calls=128):
    """(harmonic-protocol ms per call, dominant-kernel ms, kernel name)."""
    t = harmonic_runs(A, xd, yd, runs, calls)
    k_ms, _, kern = A.time_spmv(xd, yd, calls)
    return t, k_ms, kern


def suite(args):
    import torch
    import paper_1711_05487_amd as pkg
    import synth
    from paper_1711_05487_amd import learn

    torch.cuda.set_device(0)
    learn.install()
    _, wm, wrp, wcol, wval = synth.laplacian2d(64)  # load the selection kernels once
    W = pkg.CsrMatrix(wrp, wcol, wval, n_cols=wm)
    for mode in ("learned", "profile"):
        W.select(mode)
    W.close()
    triad = pkg.triad(1 << 30, 5) / 1e9
    triad_mall = pkg.triad(48 << 20, 20) / 1e9
    emit({"case": "triad", "hbm_gbs": round(triad, 1), "mall_gbs": round(triad_mall, 1),
          "device": torch.cuda.get_device_name(0)})

    workloads = [
        ("C1", "2-D 5-point Laplacian 100^2", lambda: synth.laplacian2d(100), 101),
        ("C2", "27-point stencil 128^3", lambda: synth.stencil27(128), 203),
        ("C3a", "R-MAT scale 22, edge factor 16", lambda: synth.rmat(22), 303),
        ("C3a-perm", "R-MAT scale 22, seeded symmetric permutation",
         lambda: permuted(synth.rmat(22)), 303),
        ("C3b", "uniform random 2^20 x 16", lambda: synth.uniform_random(1 << 20, 16), 403),
    ]
    for tag, desc, gen, xseed in workloads:
        log(f"{tag}: generating {desc}")
        n, m, rp, col, val = gen()
        nnz = len(col)
        x = synth.vector(m, xseed)
        chk = GpuCheck(pkg, rp, col, val, x, m)
        xd = chk.x
        yd = torch.empty(n, dtype=torch.float64, device="cuda")
        A = pkg.CsrMatrix(rp, col, val, n_cols=m)
        plain = A.select("plain")
        t_plain, k_plain, kern_plain = time_plan(A, xd, yd)
        for mode in ("plain", "learned", "profile", "exhaustive"):
            log(f"{tag}: {mode}")
            info = plain if mode == "plain" else A.select(mode)
            t, k_ms, kern = (t_plain, k_plain, kern_plain) if mode == "plain" else time_plan(A, xd, yd)
            A.spmv(xd, yd)
            torch.cuda.synchronize()
            ok = chk.f64_ok(yd)
            fb = info["format_bytes"]
            t_pre = info["t_select_ms"] + info["t_prep_ms"]
            emit({"case": tag, "workload": f"{desc} (N={n:,}, NNZ={nnz:,})", "selector": mode,
                  "opts": [nm for bit, nm in pkg.OPT_NAMES.items() if info["opts"] & bit],
                  "variant_id": info["variant_id"], "merge_items": info["merge_items"],
                  "lanes_per_row": info["lanes_per_row"], "delta_bits": info["delta_bits"],
                  "ms": round(t, 5), "kernel_ms": round(k_ms, 5), "kernel": kern,
                  "format_bytes": fb, "gbs": round(fb / (t * 1e-3) / 1e9, 1),
                  "kernel_gbs": round(fb / (k_ms * 1e-3) / 1e9, 1),
                  "pct_hbm_peak": round(100 * fb / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 2),
                  "pct_triad": round(100 * fb / (t * 1e-3) / 1e9 / triad, 2),
                  "gflops": round(2 * nnz / (t * 1e-3) / 1e9, 2),
                  "speedup_vs_plain": round(t_plain / t, 4),
                  "select_ms": round(info["t_select_ms"], 3), "prep_ms": round(info["t_prep_ms"], 3),
                  "select_cost_in_plain_spmvs": round(info["t_select_ms"] / t_plain, 2),
                  "n_iters_min": (None if mode == "plain" or n_iters_min(t_pre, t_plain, t) is None
                                  else round(n_iters_min(t_pre, t_plain, t), 1)),
                  "classes": info["classes"], "parity_ok": ok})
        if tag == "C3b":
            # cold runs: a 1 GiB write between calls evicts L2 and the MALL
            info = A.select("learned")
            flush = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
            ts = []
            for _ in range(20):
                flush.zero_()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                A.spmv(xd, yd)
                e1.record()
                e1.synchronize()
                ts.append(e0.elapsed_time(e1))
            del flush
            t = float(np.mean(ts[2:]))
            fb = info["format_bytes"]
            emit({"case": tag, "selector": "learned", "cold": True, "ms": round(t, 5),
                  "gbs": round(fb / (t * 1e-3) / 1e9, 1)})
        A.close()
        del chk

    # C4: value storage x index format on C1 and C2 (FP32 accumulation for f32/bf16)
    for tag, desc, gen, xseed in workloads[:2]:
        n, m, rp, col, val = gen()
        x = synth.vector(m, xseed)
        chk = GpuCheck(pkg, rp, col, val, x, m)
        x32 = chk.x.float()
        for storage in ("f64", "f32", "bf16"):
            A = pkg.CsrMatrix(rp, col, val, n_cols=m, storage=storage)
            xs = chk.x if storage == "f64" else x32
            ys = torch.empty(n, dtype=xs.dtype, device="cuda")
            for index in ("int32", "delta"):
                # merge-path tiles with int32 columns, then with the MB
                # remedy's codes (window ranks or offsets, whichever applies)
                opts = pkg.OPT_MERGE | (pkg.OPT_PREFETCH if index == "int32" else pkg.OPT_DELTA)
                info = A.select("forced", forced_opts=opts)
                if index == "delta" and info["delta_bits"] == 32:
                    continue  # not eligible
                t, k_ms, kern = time_plan(A, xs, ys)
                A.spmv(xs, ys)
                torch.cuda.synchronize()
                mx, p99 = chk.rel_errors(ys)
                fb = info["format_bytes"]
                emit({"case": "C4", "config": tag, "storage": storage,
                      "index": ("int32" if info["delta_bits"] == 32 else
                                f"window{info['delta_bits']}" if info["window_codes"]
                                else f"delta{info['delta_bits']}")
                      + (" runs" if info["window_codes"] == 2 else ""),
                      "merge_items": info["merge_items"],
                      "opts": [nm for bit, nm in pkg.OPT_NAMES.items() if info["opts"] & bit],
                      "ms": round(t, 5), "kernel_ms": round(k_ms, 5), "format_bytes": fb,
                      "gbs": round(fb / (t * 1e-3) / 1e9, 1),
                      "max_rel_err_vs_gpu_f64": mx, "p99_rel_err_vs_gpu_f64": p99})
            A.close()
        del chk

    c5_batch(pkg, synth, torch)


def c5_batch(pkg, synth, torch):
    """C5-batch: 512 matrices, one graph-captured persistent launch against
    512 separate launches, each matrix with its own selected plan."""
    log("C5-batch: generating 512 matrices")
    mats = [synth.batch_matrix(i) for i in range(512)]
    hs, xs, ys, fbytes, rows, nnz = [], [], [], 0, 0, 0
    for k, (_, (n, m, rp, col, val)) in enumerate(mats):
        A = pkg.CsrMatrix(rp, col, val, n_cols=m)
        fbytes += A.select("learned")["format_bytes"]
        rows += n
        nnz += len(col)
        hs.append(A)
        xs.append(torch.from_numpy(synth.vector(m, 602 + k)).cuda())
        ys.append(torch.empty(max(n, 1), dtype=torch.float64, device="cuda"))
    pkg.spmv_batched(hs, xs, ys)  # plans, tiles and the graph are built here
    torch.cuda.synchronize()
    ref = [y.clone() for y in ys]

    def timed(fn, reps=20):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    t_batch = timed(lambda: pkg.spmv_batched(hs, xs, ys))
    batch_ok = all(torch.equal(a, b) for a, b in zip(ys, ref))

    def separate():
        for A, x, y in zip(hs, xs, ys):
            A.spmv(x, y)

    t_sep = timed(separate)
    emit({"case": "C5-batch", "matrices": len(hs), "rows": rows, "nnz": nnz,
          "format_bytes": fbytes, "batched_ms": round(t_batch, 4), "separate_ms": round(t_sep, 4),
          "batched_gnnz_s": round(nnz / (t_batch * 1e-3) / 1e9, 1),
          "batched_gbs": round(fbytes / (t_batch * 1e-3) / 1e9, 1),
          "separate_gbs": round(fbytes / (t_sep * 1e-3) / 1e9, 1),
          "speedup": round(t_sep / t_batch, 3), "replay_identical": batch_ok})
    for A in hs:
        A.close()


def batch_only():
    import torch
    import paper_1711_05487_amd as pkg
    import synth
    from paper_1711_05487_amd import learn

    torch.cuda.set_device(0)
    learn.install()
    c5_batch(pkg, synth, torch)


# ---------------------------------------------------------------------------
# --amortize: what the selection costs against what it saves (Sec. IV-D)
# ---------------------------------------------------------------------------

# (label, csr_select mode, config overrides): the optimizers of Table V. The
# trivial optimizers time every candidate (the baseline and the 5 single
# remedies, or the whole 16-entry catalogue) and keep the fastest.
OPTIMIZERS = [
    ("plain", "plain", {}),
    ("trivial-single", "exhaustive", {"exhaustive_set": 1}),
    ("trivial-combined", "exhaustive", {"exhaustive_set": 0}),
    ("profile-guided", "profile", {}),
    ("feature-guided (tree)", "tree", {}),
    ("feature-guided (MLP)", "learned", {}),
]


def pcg(A, b, dinv, tol=1e-8, max_iter=4000, check_every=8):
    """Jacobi-preconditioned conjugate gradients around the library's SpMV.
    The vector updates are the same torch operations for every plan (t_other
    of Eq. (2)); the residual norm is read back every `check_every` steps.
    Returns (x, iterations)."""
    import torch
    x = torch.zeros_like(b)
    r = b.clone()
    z = dinv * r
    p = z.clone()
    q = torch.empty_like(b)
    rz = torch.dot(r, z)
    stop = tol * float(torch.linalg.vector_norm(b))
    it = 0
    while it < max_iter:
        A.spmv(p, q)
        alpha = rz / torch.dot(p, q)
        x.add_(alpha * p)
        r.sub_(alpha * q)
        it += 1
        if it % check_every == 0 and float(torch.linalg.vector_norm(r)) <= stop:
            break
        torch.mul(dinv, r, out=z)
        rz_new = torch.dot(r, z)
        p.mul_(rz_new / rz).add_(z)
        rz = rz_new
    return x, it


def select_timed(pkg, A, mode, over):
    """Host wall time of csr_select (features or probes, decision, format
    preparation): the t_pre of Eq. (2)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = A.select(mode, **over)
    torch.cuda.synchronize()
    return info, (time.perf_counter() - t0) * 1e3


def amortize(args):
    import torch
    import paper_1711_05487_amd as pkg
    import synth
    from paper_1711_05487_amd import learn

    from paper_1711_05487_amd import tree
    torch.cuda.set_device(0)
    learn.install()
    tree.install()
    # load every selection kernel once (a process cost, not a per-matrix one)
    _, wm, wrp, wcol, wval = synth.laplacian2d(64)
    W = pkg.CsrMatrix(wrp, wcol, wval, n_cols=wm)
    for _, mode, over in OPTIMIZERS:
        W.select(mode, **over)
    W.close()

    # 1. Table V: N_iters,min over held-out matrices of the selector's suite
    recs = learn.read_labels(os.path.join(ROOT, "paper_1711_05487_amd", "weights",
                                          "labels_mi355x.jsonl"))
    _, test = learn.split(recs)
    big = [r for r in test if r["nnz"] >= 100_000]
    step = max(1, len(big) // max(1, args.amortize_matrices))
    picks = big[::step][:args.amortize_matrices]
    per_opt = {lab: [] for lab, _, _ in OPTIMIZERS[1:]}
    for k, r in enumerate(picks):
        name, (n, m, rp, col, val) = synth.suite_matrix(r["index"])
        x = torch.from_numpy(synth.vector(m, 602 + r["index"])).cuda()
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        times = {}
        for lab, mode, over in OPTIMIZERS:
            A = pkg.CsrMatrix(rp, col, val, n_cols=m)
            info, t_pre = select_timed(pkg, A, mode, over)
            t_spmv, _, _ = time_plan(A, x, y, runs=3, calls=64)
            times[lab] = (t_pre, t_spmv, info)
            A.close()
        t_plain = times["plain"][1]
        for lab, _, _ in OPTIMIZERS[1:]:
            t_pre, t_spmv, info = times[lab]
            nim = n_iters_min(t_pre, t_plain, t_spmv)
            per_opt[lab].append(nim)
            emit({"case": "table5", "matrix": name, "index": r["index"], "nnz": int(len(col)),
                  "optimizer": lab, "t_pre_ms": round(t_pre, 3), "t_spmv_ms": round(t_spmv, 5),
                  "t_plain_ms": round(t_plain, 5),
                  "speedup_vs_plain": round(t_plain / t_spmv, 4),
                  "opts": [nm for bit, nm in pkg.OPT_NAMES.items() if info["opts"] & bit],
                  "n_iters_min": None if nim is None else round(nim, 1)})
        log(f"table5 {k + 1}/{len(picks)} {name}")
    for lab, vals in per_opt.items():
        fin = [v for v in vals if v is not None]
        emit({"case": "table5-summary", "optimizer": lab, "matrices": len(vals),
              "never_amortized": len(vals) - len(fin),
              "n_iters_best": round(min(fin), 1) if fin else None,
              "n_iters_avg": round(float(np.mean(fin)), 1) if fin else None,
              "n_iters_median": round(float(np.median(fin)), 1) if fin else None,
              "n_iters_worst": round(max(fin), 1) if fin else None})

    # 2. Conjugate-gradient solves on SPD systems, end to end
    systems = [
        ("lap3d_128", "7-point 3-D Laplacian 128^3", lambda: synth.laplacian3d(128)),
        ("spd27_128", "SPD 27-point stencil 128^3 (symmetric, diagonally dominant)",
         lambda: synth.spd_stencil27(128)),
        ("lap2d_1024", "5-point 2-D Laplacian 1024^2", lambda: synth.laplacian2d(1024)),
    ]
    for tag, desc, gen in systems:
        n, m, rp, col, val = gen()
        rows = np.repeat(np.arange(n), np.diff(rp))
        diag = np.zeros(n)
        diag[rows[col == rows]] = val[col == rows]
        dinv = torch.from_numpy(1.0 / diag).cuda()
        x_true = torch.from_numpy(synth.vector(m, 901)).cuda()
        P = pkg.CsrMatrix(rp, col, val, n_cols=m)
        b = P.spmv(x_true)
        P.close()
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        base = None
        for lab, mode, over in OPTIMIZERS:
            A = pkg.CsrMatrix(rp, col, val, n_cols=m)
            info, t_pre = select_timed(pkg, A, mode, over)
            t_spmv, _, _ = time_plan(A, x_true, y, runs=3, calls=64)
            pcg(A, b, dinv, max_iter=16)  # warm the solver's own kernels
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            xs, it = pcg(A, b, dinv)
            e1.record()
            torch.cuda.synchronize()
            t_solve = e0.elapsed_time(e1)
            err = float(torch.linalg.vector_norm(xs - x_true) / torch.linalg.vector_norm(x_true))
            if base is None:
                base = (t_spmv, t_solve)
            nim = None if lab == "plain" else n_iters_min(t_pre, base[0], t_spmv)
            emit({"case": "cg", "system": tag, "workload": f"{desc} (N={n:,}, NNZ={len(col):,})",
                  "optimizer": lab,
                  "opts": [nm for bit, nm in pkg.OPT_NAMES.items() if info["opts"] & bit],
                  "window_codes": bool(info["window_codes"]), "iterations": it,
                  "rel_error": err, "t_pre_ms": round(t_pre, 3), "t_spmv_ms": round(t_spmv, 5),
                  "t_solve_ms": round(t_solve, 3), "t_total_ms": round(t_pre + t_solve, 3),
                  "solve_speedup_vs_plain": round(base[1] / t_solve, 4),
                  "total_speedup_vs_plain": round(base[1] / (t_pre + t_solve), 4),
                  "n_iters_min": None if nim is None else round(nim, 1)})
            A.close()
        log(f"cg {tag} done")


# ---------------------------------------------------------------------------
# --irregular: the plans of the gather-bound configurations, for counter runs
# ---------------------------------------------------------------------------

def irregular(args):
    """R-MAT scale 22 and uniform 2^20 x 16 under plain CSR, the merge path
    and (uniform) the column-blocked merge path: `args.steps` calls each, one
    JSON line per plan with the algorithmic bytes of one call."""
    import torch
    import paper_1711_05487_amd as pkg
    import synth
    torch.cuda.set_device(0)
    M, P = pkg.OPT_MERGE, pkg.OPT_PREFETCH
    one = {"split_row_blocks": 0}  # tiles with split rows: a single pass
    rmat_plans = [("plain", 0, {}), ("merge, one pass", M, one),
                  ("prefetch+merge, one pass", M | P, one),
                  ("merge (column blocks over row lists)", M, {})]
    cases = [("C3a", "R-MAT scale 22, edge factor 16", lambda: synth.rmat(22), 303, rmat_plans),
             ("C3a-perm", "R-MAT scale 22, seeded symmetric permutation",
              lambda: permuted(synth.rmat(22)), 303, rmat_plans),
             ("C3b", "uniform random 2^20 x 16", lambda: synth.uniform_random(1 << 20, 16), 403,
              [("plain", 0, {}), ("merge", M, {}),
               ("prefetch+merge (column blocks)", M | P, {})])]
    for tag, desc, gen, xseed, plans in cases:
        n, m, rp, col, val = gen()
        x = torch.from_numpy(synth.vector(m, xseed)).cuda()
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        A = pkg.CsrMatrix(rp, col, val, n_cols=m)
        for name, opts, over in plans:
            info = A.select("forced", forced_opts=opts, **over)
            for _ in range(args.warmup):
                A.spmv(x, y)
            torch.cuda.synchronize()
            for _ in range(args.steps):
                A.spmv(x, y)
            torch.cuda.synchronize()
            k_ms, _, kern = A.time_spmv(x, y, 20)
            emit({"case": tag, "workload": f"{desc} (N={n:,}, NNZ={len(col):,})", "plan": name,
                  "kernel": kern, "column_blocks": info["column_blocks"],
                  "format_bytes": info["format_bytes"], "kernel_ms": round(k_ms, 5),
                  "calls": args.steps})
        A.close()


# --partitions: the partition-aware ML test (proposed with the results of
# Sec. IV-C) against the whole-matrix test of Fig. 4
def partitions(args):
    """Per matrix: the whole-matrix P_ML / P_CSR, the largest partition ratio
    (256 partitions) and the flagged partitions; the profile-guided plan's
    kernel time without and with the partition test, with ML forced on and
    off (the remedy's value), the learned plan's and plain CSR's."""
    import torch
    import paper_1711_05487_amd as pkg
    import synth
    from paper_1711_05487_amd import learn
    torch.cuda.set_device(0)
    learn.install()
    cases = []
    for lg in (21, 22):
        for frac in (1 / 256, 1 / 128, 1 / 64, 1 / 32):
            cases.append((f"localized 2^{lg} x 16, {frac * 100:.2f}% irregular rows",
                          lambda lg=lg, frac=frac: synth.localized_irregular(1 << lg, 16, frac, 811)))
    for i in range(3, 2000, 37):
        if i % 5 != 0:  # the stencil family has no irregular gathers
            cases.append((f"suite {i}", lambda i=i: synth.suite_matrix(i)[1]))
    for name, gen in cases:
        n, m, rp, col, val = gen()
        x = torch.from_numpy(synth.vector(m, 3)).cuda()
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        A = pkg.CsrMatrix(rp, col, val, n_cols=m)

        def timed():
            return round(A.time_spmv(x, y, 30)[0] * 1000, 2)
        A.select("plain")
        t_plain = timed()
        ia = A.select("profile")
        t_a = timed()
        ib = A.select("profile", ml_partitions=256)
        t_b = timed()
        A.select("profile", t_ml=0.0)
        t_on = timed()
        A.select("profile", t_ml=1e9)
        t_off = timed()
        A.select("learned")
        t_l = timed()
        emit({"matrix": name, "n": n, "nnz": int(rp[-1]),
              "ml_whole": round(ia["p_ml"] / ia["p_csr"], 3),
              "ml_part_max": round(ib["ml_part_max"], 3), "parts": ib["ml_partitions"],
              "flagged": ib["ml_parts_flagged"], "classes": ia["classes"],
              "classes_partitions": ib["classes"], "us_plain": t_plain, "us_profile": t_a,
              "us_profile_partitions": t_b, "us_ml_on": t_on, "us_ml_off": t_off,
              "us_learned": t_l})
        A.close()


if __name__ == "__main__":
    main()

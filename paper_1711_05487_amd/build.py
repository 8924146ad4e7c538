"""Build libcsrspmv.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_1711_05487_amd.build          # incremental
    python -m paper_1711_05487_amd.build --force  # rebuild everything
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libcsrspmv.so")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]

# (object name, source, extra defines)
UNITS = [
    ("api", "api.hip", []),
    ("select", "select.hip", []),
    ("k_prep", "k_prep.hip", []),
    ("k_features", "k_features.hip", []),
    ("k_mlp", "k_mlp.hip", []),
    ("learn", "learn.hip", []),
    ("batch", "batch.hip", []),
    ("k_batched_f64", "k_batched.hip", ["-DCSR_STORAGE=0"]),
    ("k_batched_f32", "k_batched.hip", ["-DCSR_STORAGE=1"]),
    ("k_batched_bf16", "k_batched.hip", ["-DCSR_STORAGE=2"]),
    ("k_long_f64", "k_long.hip", ["-DCSR_STORAGE=0"]),
    ("k_long_f32", "k_long.hip", ["-DCSR_STORAGE=1"]),
    ("k_long_bf16", "k_long.hip", ["-DCSR_STORAGE=2"]),
    ("k_rowsplit_f64", "k_rowsplit.hip", ["-DCSR_STORAGE=0"]),
    ("k_rowsplit_f32", "k_rowsplit.hip", ["-DCSR_STORAGE=1"]),
    ("k_rowsplit_bf16", "k_rowsplit.hip", ["-DCSR_STORAGE=2"]),
    ("k_merge_f64", "k_merge.hip", ["-DCSR_STORAGE=0"]),
    ("k_merge_f32", "k_merge.hip", ["-DCSR_STORAGE=1"]),
    ("k_merge_bf16", "k_merge.hip", ["-DCSR_STORAGE=2"]),
]


def _headers_mtime() -> float:
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    hs.append(os.path.join(ROOT, "include", "csrspmv.h"))
    return max(os.path.getmtime(h) for h in hs)


def _compile(unit, force):
    name, src, defs = unit
    obj = os.path.join(BUILD, name + ".o")
    srcp = os.path.join(CSRC, src)
    if (not force and os.path.exists(obj)
            and os.path.getmtime(obj) >= max(os.path.getmtime(srcp), _headers_mtime())):
        return obj, False
    cmd = [HIPCC, *FLAGS, *defs, "-c", srcp, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj, True


def build(force: bool = False, jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        res = list(ex.map(lambda u: _compile(u, force), UNITS))
    objs = [o for o, _ in res]
    changed = any(c for _, c in res)
    if force or changed or not os.path.exists(OUT):
        tmp = OUT + f".tmp{os.getpid()}"
        cmd = [HIPCC, "-shared", "--offload-arch=gfx950", "-o", tmp, *objs]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stderr}")
        os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(force="--force" in sys.argv))

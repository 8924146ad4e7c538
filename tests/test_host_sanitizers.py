"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(host pass only; the device code is built as usual), run on the CPU: every
entry point that does its work before reaching a GPU is called with valid and
invalid arguments in a child process with the ASan runtime preloaded, which
aborts on the first report (memory error or undefined behaviour)."""
import os
import subprocess
import sys
import textwrap

import pytest

from paper_1711_05487_amd import build as hipbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent(r'''
    import ctypes, sys
    sys.path.insert(0, sys.argv[2])
    import paper_1711_05487_amd as pkg
    L = ctypes.CDLL(sys.argv[1])
    P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    L.csr_status_str.restype = ctypes.c_char_p
    L.csr_last_error.restype = ctypes.c_char_p
    cfg = pkg.Config()
    L.csr_config_default(ctypes.byref(cfg))
    assert cfg.t_ml == 1.0 and cfg.remedy_map == 1 and cfg.timing_calls == 32
    for s in range(-1, 9):
        assert L.csr_status_str(s)
    h = P()
    # csr_create: argument errors are caught before any device work
    assert L.csr_create(None, 4, 4, 4, P(8), P(8), P(8), 0, None) == 1
    assert L.csr_create(ctypes.byref(h), -1, 4, 4, P(8), P(8), P(8), 0, None) == 1
    assert L.csr_create(ctypes.byref(h), 4, 4, i64(1 << 31), P(8), P(8), P(8), 0, None) == 5
    assert L.csr_create(ctypes.byref(h), 4, 4, 4, P(8), None, P(8), 0, None) == 1
    assert L.csr_create(ctypes.byref(h), 4, 4, 4, P(8), P(8), P(8), 7, None) == 1
    assert b"storage" in L.csr_last_error()
    L.csr_destroy(None)
    assert L.csr_spmv(None, P(8), P(8), None) == 1
    assert L.csr_select(None, 0, None, None, None) == 1
    assert L.csr_inspect(None, None, None) == 1
    assert L.csr_query(None, None, None, None, None, None) == 1
    assert L.csr_debug_copy(None, 0, None, 0, None, None) == 1
    assert L.csr_spmv_batched(-1, None, None, None, None) == 1
    assert L.csr_spmv_batched(0, None, None, None, None) == 0
    assert L.csr_spmv_noalloc(-1, 4, i64(0), P(8), None, None, P(8), P(64), None) == 1
    assert L.csr_spmv_noalloc(4, 4, i64(4), P(8), P(8), P(8), P(4096), P(4096 + 8), None) == 1
    assert L.csr_spmv_noalloc(0, 0, i64(0), P(8), None, None, None, None, None) == 0
    assert L.csr_triad(sz(16), 1, None, None) == 1
    assert L.csr_debug_triad(P(16), P(32), P(48), i64(3), ctypes.c_double(1.0), 0, None) == 1
    assert L.csr_debug_triad(P(16), P(32), P(48), i64(4), ctypes.c_double(1.0), 2, None) == 1
    b, n, a = i64(), i64(), i64()
    assert L.csr_debug_alloc(1, i64(2), i64(3), ctypes.byref(b), ctypes.byref(n), ctypes.byref(a)) == 0
    assert L.csr_debug_alloc(0, i64(0), i64(0), None, None, ctypes.byref(a)) == 0 and a.value == 0
    assert L.csr_debug_alloc(1, i64(-1), i64(0), None, None, None) == 1
    assert L.csr_debug_alloc(1, i64(0), i64(0), None, None, None) == 0
    # the decision tree's validation (host only)
    f = (i32 * 3)(0, -1, -1); t = (ctypes.c_double * 3)(0.5, 0, 0)
    lt = (i32 * 3)(1, 0, 0); rt = (i32 * 3)(2, 0, 0); v = (i32 * 3)(0, 3, 5)
    assert L.csr_tree_load(3, f, t, lt, rt, v) == 0
    bad = (i32 * 3)(0, 0, 0)   # a child that does not follow its parent
    assert L.csr_tree_load(3, f, t, bad, rt, v) == 1
    v16 = (i32 * 3)(0, 3, 16)  # a class mask out of range
    assert L.csr_tree_load(3, f, t, lt, rt, v16) == 1
    f17 = (i32 * 3)(17, -1, -1)
    assert L.csr_tree_load(3, f17, t, lt, rt, v) == 1
    assert L.csr_tree_unload() == 0
    # run-time compilation of the merge kernel (host string handling + hipRTC)
    need = sz()
    assert L.csr_jit_compile(0, 768, 0, 1, 1, None, sz(0), ctypes.byref(need)) == 0
    buf = ctypes.create_string_buffer(need.value)
    assert L.csr_jit_compile(0, 768, 0, 1, 1, buf, need, ctypes.byref(need)) == 0
    assert buf.raw[:4] == b"\x7fELF"
    assert L.csr_jit_compile(1, 1280, 0, 0, 0, None, sz(0), ctypes.byref(need)) == 0
    assert L.csr_jit_compile(0, 700, 0, 1, 1, None, sz(0), ctypes.byref(need)) == 1
    assert L.csr_jit_compile(0, 768, 9, 1, 1, None, sz(0), ctypes.byref(need)) == 1
    print("sanitized host checks passed")
''')


@pytest.mark.timeout(900)
def test_host_code_under_asan_and_ubsan():
    lib = hipbuild.build(sanitize=True)
    env = dict(os.environ)
    env["LD_PRELOAD"] = hipbuild.sanitizer_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env.pop("PYTHONPATH", None)
    r = subprocess.run([sys.executable, "-c", CHILD, lib, ROOT], capture_output=True, text=True,
                       env=env, timeout=600)
    msg = r.stdout[-3000:] + r.stderr[-6000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, msg
    assert r.returncode == 0, msg
    assert "sanitized host checks passed" in r.stdout, msg

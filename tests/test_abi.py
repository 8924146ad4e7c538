"""Host-side checks of the C-ABI library: it loads, exports every entry point
declared in include/csrspmv.h, and rejects bad arguments before touching the
device. No compute call is made here (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_1711_05487_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "csrspmv.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(csr_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = pkg.lib()
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(pkg.EXPORTS)


def test_status_strings_and_defaults():
    L = pkg.lib()
    for k, name in enumerate(pkg.STATUS):
        assert L.csr_status_str(k).decode() == name
    c = pkg.default_config()
    assert (c.t_ml, c.t_imb, c.t_mb, c.remedy_map, c.split_row_blocks) == (1.0, 1.0, 0.5, 1, 1)
    assert c.ood_z == 4.0
    assert c.long_row_factor == 32.0 and c.long_row_floor == 4096 and c.timing_calls == 32


def test_argument_errors_before_device_work():
    L = pkg.lib()
    P = ctypes.c_void_p
    h = P()
    assert L.csr_create(None, 1, 1, 0, P(1), None, None, 0, None) == 1
    assert L.csr_create(ctypes.byref(h), -1, 1, 0, P(1), None, None, 0, None) == 1
    assert h.value is None
    assert L.csr_create(ctypes.byref(h), 2, 2, 1 << 31, P(1), P(1), P(1), 0, None) == 5
    assert L.csr_create(ctypes.byref(h), 2, 2, (1 << 31) - 4095, P(1), P(1), P(1), 0, None) == 5
    assert L.csr_create(ctypes.byref(h), 2, 2, 3, P(1), None, P(1), 0, None) == 1
    assert L.csr_create(ctypes.byref(h), 2, 2, 3, P(1), P(1), P(1), 7, None) == 1
    assert L.csr_spmv(None, P(1), P(2), None) == 1
    assert L.csr_select(None, 0, None, None, None) == 1
    assert L.csr_inspect(None, None, None) == 1
    assert L.csr_query(None, None, None, None, None, None) == 1
    assert L.csr_spmv_batched(-1, None, None, None, None) == 1
    assert L.csr_triad(16, 1, None, None) == 1
    assert b"NULL" in L.csr_last_error() or len(L.csr_last_error()) > 0
    L.csr_destroy(None)  # accepted


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(pkg, "_lib", None)
    monkeypatch.setattr(pkg, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        pkg.lib()


def test_struct_layout_matches_header(tmp_path):
    """The ctypes mirrors of csr_config_t, csr_plan_info_t and csr_features_t
    have the C header's size and field offsets (a C program compiled with
    the header prints them)."""
    structs = {"csr_config_t": pkg.Config, "csr_plan_info_t": pkg.PlanInfo,
               "csr_features_t": pkg.Features}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "csrspmv.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_classify_matches_oracle_rule():
    """The library's profile-guided rule and class -> remedy map (host code,
    no GPU) against the oracle's on random bounds and thresholds."""
    import numpy as np
    import oracle
    import synth
    rng_u = lambda s, n: synth.u01(s, 0, np.arange(n, dtype=np.uint64))
    n = 4000
    P = 10.0 ** (9 + 3 * rng_u(11, 6 * n).reshape(n, 6))
    T = 0.5 + 2.0 * rng_u(12, 3 * n).reshape(n, 3)
    for k in range(n):
        cfg = pkg.default_config()
        cfg.t_ml, cfg.t_imb, cfg.t_mb = T[k]
        cfg.remedy_map = k % 2
        has_long = bool(k % 3 == 0)
        cls, opts = pkg.classify(P[k], has_long, config=cfg)
        want = oracle.classify(*P[k], t_ml=T[k, 0], t_imb=T[k, 1], t_mb=T[k, 2])
        assert cls == want, (k, P[k], T[k])
        assert opts == oracle.remedies(want, has_long, k % 2)
    with pytest.raises(pkg.CsrError):
        pkg.classify([1.0, 1.0, 1.0, 0.0, 1.0, 1.0], False)
    with pytest.raises(pkg.CsrError):
        pkg.classify([1.0] * 6, False, remedy_map=2)

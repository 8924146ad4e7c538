"""Run-time specialization of the merge-path kernel (the paper's
just-in-time code generation, Sec. IV-D) on the host: csr_jit_compile needs
no GPU. The compiled instance of a prebuilt tile size is instruction for
instruction the library's own kernel, run-time sizes compile without packed
FP32 instructions, and instances that cannot exist are refused.

The run-time compiler is whichever hipRTC the process has loaded: the
system ROCm's in a process without PyTorch (the compiler of the prebuilt
kernels), PyTorch's own copy once torch is imported (as in every GPU run).
The instruction comparison therefore runs in a process without torch, and
the packed-FP32 check in one with torch loaded first."""
import os
import re
import subprocess
import sys

import pytest

import paper_1711_05487_amd as pkg
from paper_1711_05487_amd import build as B

OBJDUMP = "/opt/rocm/llvm/bin/llvm-objdump"
W8, D16, D8 = 3, 1, 2


def kernel_lines(path):
    """(symbol, instructions) of the one k_merge kernel in a code object (or
    of the instance whose mangled template arguments contain `tag`)."""
    d = subprocess.run([OBJDUMP, "-d", "--no-show-raw-insn", "--no-leading-addr", path],
                       capture_output=True, text=True, check=True).stdout
    out = {}
    for block in re.split(r"\n(?=\S.*>:\n)", d):
        head = block.split("\n", 1)[0]
        if "k_merge" not in head:
            continue
        lines = [re.sub(r"<[^>]*>", "", l.split("//")[0]).strip() for l in block.split("\n")[1:]]
        lines = [l for l in lines if l and not l.startswith(";")]
        # zero words after the last branch are padding between functions
        # (disassembled as v_cndmask, or elided as "...")
        while lines and lines[-1] in ("v_cndmask_b32_e32 v0, s0, v0, vcc", "..."):
            lines.pop()
        out[head] = lines
    return out


@pytest.mark.parametrize("args", [
    dict(merge_items=768),
    dict(merge_items=768, streaming=False, row_aligned=False),
    dict(merge_items=1536, index_mode=D16),
    dict(merge_items=2048, index_mode=W8),
    dict(merge_items=2048, storage="bf16", index_mode=D8),
    dict(merge_items=1280, storage="f32"),
])
def test_compiles_without_packed_fp32(args, tmp_path):
    import torch  # noqa: F401  (its hipRTC, the one GPU runs compile with)
    code = pkg.jit_compile(**args)
    assert code[:4] == b"\x7fELF"
    p = tmp_path / "k.co"
    p.write_bytes(code)
    kernels = kernel_lines(str(p))
    assert len(kernels) == 1
    (head, lines), = kernels.items()
    ipt = args["merge_items"] // 64
    assert f"k_mergeILi{ipt}E" in head
    assert len(lines) > 100
    assert not [l for l in lines if re.match(r"v_pk_(fma|mul|add)_f32", l)]


@pytest.mark.parametrize("args", [
    dict(merge_items=640),                                  # not a multiple of 256
    dict(merge_items=4096),                                 # above 2048
    dict(merge_items=768, index_mode=W8, row_aligned=False),
    dict(merge_items=768, index_mode=D8),                   # 12 code bytes per lane
    dict(merge_items=1536, index_mode=W8),                  # 24 code bytes per lane
    dict(merge_items=768, storage=7),
    dict(merge_items=768, index_mode=9),
])
def test_impossible_instances_refused(args):
    with pytest.raises(pkg.CsrError):
        pkg.jit_compile(**args)


def test_same_instructions_as_the_prebuilt_kernel(tmp_path):
    """k_merge<8, true, false, 3, true> (FP64, L = 512, window codes, row-
    aligned tiles) compiled at run time against the same instance compiled
    ahead of time with the library's flags."""
    aot = tmp_path / "aot.co"
    flags = [f for f in B.FLAGS if f != "-fPIC"]
    subprocess.run([B.HIPCC, *flags, "-DCSR_STORAGE=0", "--cuda-device-only",
                    "--no-gpu-bundle-output", "-c", os.path.join(B.CSRC, "k_merge.hip"),
                    "-o", str(aot)], check=True, capture_output=True)
    jit = tmp_path / "jit.co"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    prog = ("import sys; import paper_1711_05487_amd as pkg; "
            "assert 'torch' not in sys.modules; "
            f"open({str(jit)!r}, 'wb').write(pkg.jit_compile(merge_items=512, index_mode={W8}))")
    subprocess.run([sys.executable, "-c", prog], check=True, cwd=root, capture_output=True)
    want = [v for k, v in kernel_lines(str(aot)).items() if "k_mergeILi8ELb1ELb0ELi3ELb1E" in k]
    got = list(kernel_lines(str(jit)).values())
    assert len(want) == 1 and len(got) == 1
    assert len(want[0]) > 500
    assert got[0] == want[0]

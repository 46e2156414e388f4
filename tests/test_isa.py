"""The gfx950 code of the library, read back from the built libht.so: the vote arithmetic must be
one rounding per operation, so the fill kernels may hold no fused float multiply-add, and the
per-hit preparation may hold only the fused operations of its correctly rounded square root and
division (the very sequences that tests/test_gpu_unary.py checks over every binary32 input).
Nothing may use packed FP32 arithmetic. Needs no GPU: objcopy, clang-offload-bundler and
llvm-objdump take the code object apart on the host."""
import collections
import os
import re
import shutil
import subprocess

import pytest

from paper_1507_03074_amd import binding as B

LLVM = "/opt/rocm/llvm/bin"
FUSED_F32 = re.compile(r"\bv_(pk_)?(fma|fmac|mac|mad)(_mix\w*|_f32|_legacy_f32)\w*")
PACKED_F32 = re.compile(r"\bv_pk_(add|mul|fma|mov)_f32\b")
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"


@pytest.fixture(scope="module")
def disasm(tmp_path_factory):
    from paper_1507_03074_amd import build as hbuild
    hbuild.ensure_built()  # a missing or stale library is rebuilt, never tested
    tools = [shutil.which("objcopy"), os.path.join(LLVM, "clang-offload-bundler"),
             os.path.join(LLVM, "llvm-objdump")]
    if not all(t and os.path.exists(t) for t in tools):
        pytest.skip("objcopy / ROCm LLVM tools not available")
    d = tmp_path_factory.mktemp("isa")
    fat, scratch = str(d / "fatbin"), str(d / "copy.so")
    # with no output file objcopy would rewrite the library in place, under this process's
    # own mapping of it: the rewritten copy goes to the scratch file instead
    subprocess.check_call([tools[0], "--dump-section", ".hip_fatbin=" + fat, B.LIB_PATH, scratch])
    # one offload bundle per HIP translation unit, concatenated by the linker
    data = open(fat, "rb").read()
    starts = [m.start() for m in re.finditer(re.escape(MAGIC), data)]
    assert starts, "no offload bundle in the library"
    kernels = collections.defaultdict(list)
    for k, a in enumerate(starts):
        part, co = str(d / ("bundle%d" % k)), str(d / ("gfx950_%d.co" % k))
        with open(part, "wb") as f:
            f.write(data[a:starts[k + 1] if k + 1 < len(starts) else len(data)])
        subprocess.check_call([tools[1], "--unbundle", "--type=o",
                               "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", "--input=" + part,
                               "--output=" + co])
        text = subprocess.check_output([tools[2], "-d", "--no-show-raw-insn", co], text=True)
        cur = None
        for line in text.splitlines():
            m = re.match(r"^[0-9a-f]+ <(.+)>:$", line)
            if m:
                cur = m.group(1)
                continue
            if cur and line.strip():
                kernels[cur].append(line.strip())
    return kernels


def kernel_name(mangled):
    m = re.search(r"(k_\w+?)(?:E|I[LN]|$)", mangled)
    return m.group(1) if m else mangled


def fused(lines):
    return [ln for ln in lines if FUSED_F32.search(ln)]


def test_fill_kernels_have_no_fused_float_ops(disasm):
    fills = {k: v for k, v in disasm.items() if kernel_name(k) in ("k_fill", "k_fill_atomic")}
    assert len(fills) > 100  # every fill variant is there
    for k, lines in fills.items():
        assert not fused(lines), (k, fused(lines)[:3])


def test_preparation_fuses_only_inside_sqrt_and_division(disasm):
    by_name = collections.defaultdict(list)
    for k, lines in disasm.items():
        by_name[kernel_name(k)].append(lines)
    ref = sorted(ln.split()[0] for ln in fused(by_name["k_debug_unary"][0]))
    assert ref, "the correctly rounded sqrt and division use fused steps on this target"
    for name in ("k_prep_direct", "k_prep", "k_debug_hits"):
        assert by_name[name], name
        for lines in by_name[name]:  # every variant
            got = sorted(ln.split()[0] for ln in fused(lines))
            assert got == ref, (name, got, ref)


def test_no_packed_fp32_anywhere(disasm):
    for k, lines in disasm.items():
        bad = [ln for ln in lines if PACKED_F32.search(ln)]
        assert not bad, (k, bad[:3])

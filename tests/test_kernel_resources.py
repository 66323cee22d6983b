"""Private-segment (scratch) use of the library's kernels, read from the
gfx950 code objects inside the built libradtrace.so (their metadata notes).

A kernel that keeps part of its state in per-lane scratch memory runs far
slower than one that fits its registers: a local copy of the constants indexed
by a loop counter, or a second record buffer beyond 128 VGPRs, both put the
deposit kernels there and cost them 20-35%. The kernels of every hot path must
use none; a few wide-tile and FP64 one-antenna batch variants are known to
spill a little and may not spill more.
"""
import os
import re
import shutil
import struct
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2309_03717_amd", "libradtrace.so")
LLVM = "/opt/rocm/llvm/bin"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"

# kernels allowed some scratch (bytes): wide antenna tiles, used only for short
# traces, and the FP64 one-antenna batch kernels
ALLOWED = {
    r"deposit_kernelILi\dELi\dELi\dELi[2-8]E": 128,
    r"batch_deposit_one_kernelILi0ELi[01]E": 32,
}


def code_objects(lib):
    """The gfx950 code objects of every offload bundle in the library."""
    with tempfile.TemporaryDirectory() as d:
        sec = os.path.join(d, "fatbin")
        subprocess.run([os.path.join(LLVM, "llvm-objcopy"), f"--dump-section=.hip_fatbin={sec}",
                        lib, os.path.join(d, "copy.so")], check=True, capture_output=True)
        data = open(sec, "rb").read()
    out = []
    pos = data.find(MAGIC)
    while pos >= 0:
        n = struct.unpack_from("<Q", data, pos + len(MAGIC))[0]
        q = pos + len(MAGIC) + 8
        for _ in range(n):
            off, size, tlen = struct.unpack_from("<QQQ", data, q)
            triple = data[q + 24:q + 24 + tlen].decode()
            q += 24 + tlen
            if "gfx950" in triple:
                out.append(data[pos + off:pos + off + size])
        pos = data.find(MAGIC, pos + 1)
    return out


def kernel_scratch(lib):
    res = {}
    with tempfile.TemporaryDirectory() as d:
        for i, co in enumerate(code_objects(lib)):
            path = os.path.join(d, f"co{i}")
            open(path, "wb").write(co)
            notes = subprocess.run([os.path.join(LLVM, "llvm-readelf"), "--notes", path],
                                   check=True, capture_output=True, text=True).stdout
            name = None
            for line in notes.splitlines():
                m = re.match(r"\s*\.name:\s+(\S+)", line)
                if m:
                    name = m.group(1)
                m = re.match(r"\s*\.private_segment_fixed_size:\s+(\d+)", line)
                if m and name:
                    res[name] = int(m.group(1))
                    name = None
    return res


@pytest.fixture(scope="module")
def scratch():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    for tool in ("llvm-objcopy", "llvm-readelf"):
        if not shutil.which(os.path.join(LLVM, tool)):
            pytest.skip(f"{tool} not available")
    res = kernel_scratch(LIB)
    assert len(res) > 100, "expected the kernels of every translation unit"
    return res


def test_hot_kernels_use_no_scratch(scratch):
    """Every kernel outside the allowed list keeps its state in registers."""
    spill = {k: v for k, v in scratch.items()
             if v and not any(re.search(p, k) for p in ALLOWED)}
    assert not spill, spill


def test_known_spills_do_not_grow(scratch):
    over = {k: v for k, v in scratch.items()
            for p, lim in ALLOWED.items() if re.search(p, k) and v > lim}
    assert not over, over


def test_one_antenna_deposits_present_and_clean(scratch):
    """The one-antenna deposit kernels of every formalism, precision and medium
    (the 4096-bin workloads' kernels) exist and use no scratch."""
    for f in (0, 1):
        for p in (0, 1):
            for med in (0, 1, 2, 3):
                name = f"_ZN2rt14deposit_kernelILi{f}ELi{p}ELi{med}ELi1EEEvNS_11DepositArgsE"
                assert scratch.get(name) == 0, (name, scratch.get(name))

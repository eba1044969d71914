"""Resource use of the built kernels (no GPU): read the gfx950 code objects of the compiled
sources and check that no kernel uses private (scratch) memory or spills registers.  A by-value
kernel argument indexed with a run-time value, for instance, makes every thread copy it to
scratch, which costs more than the kernel's own traffic."""
import os
import re
import subprocess
import tempfile

import pytest

from paper_2411_19588_amd import build as B

LLVM = "/opt/rocm/llvm/bin"


def _code_object(obj: str, tmp: str) -> str:
    fat = os.path.join(tmp, "fatbin")
    subprocess.run([f"{LLVM}/llvm-objcopy", f"--dump-section=.hip_fatbin={fat}", obj], check=True,
                   capture_output=True)
    co = os.path.join(tmp, "co")
    subprocess.run([f"{LLVM}/clang-offload-bundler", "--type=o", f"--targets=hipv4-amdgcn-amd-amdhsa--{B.ARCH}",
                    f"--input={fat}", f"--output={co}", "--unbundle"], check=True, capture_output=True)
    return co


def _kernels(co: str):
    notes = subprocess.run([f"{LLVM}/llvm-readelf", "--notes", co], check=True, capture_output=True, text=True).stdout
    out = []
    for block in re.split(r"\n\s+- \.", notes):
        name = re.search(r"\.name:\s+(\S+)", block)
        priv = re.search(r"\.private_segment_fixed_size:\s+(\d+)", block)
        spill = re.search(r"\.vgpr_spill_count:\s+(\d+)", block)
        if name and priv:
            out.append((name.group(1), int(priv.group(1)), int(spill.group(1)) if spill else 0))
    return out


@pytest.mark.parametrize("src", B.SOURCES)
def test_no_scratch_and_no_spills(src):
    obj = os.path.join(B.BUILD, os.path.splitext(src)[0] + ".o")
    if not (os.path.exists(obj) and os.path.exists(f"{LLVM}/clang-offload-bundler")):
        pytest.skip("build objects or LLVM tools not available")
    sections = subprocess.run([f"{LLVM}/llvm-readelf", "-S", obj], check=True, capture_output=True, text=True).stdout
    if ".hip_fatbin" not in sections:
        pytest.skip(f"{src} holds no device code")
    with tempfile.TemporaryDirectory() as tmp:
        kernels = _kernels(_code_object(obj, tmp))
    assert kernels, "no kernel metadata found"
    bad = [(n, p, s) for n, p, s in kernels if p or s]
    assert not bad, bad

"""The library's device code contains no packed float32 arithmetic.

Every HIP source is compiled to gfx950 assembly with the library's own flags
(which disable the packed-fp32-ops target feature) and the assembly is
searched for v_pk_fma_f32 / v_pk_mul_f32 / v_pk_add_f32.  Runs on the CPU
(hipcc cross-compiles)."""
from __future__ import annotations

import os
import re
import subprocess

import pytest

from paper_2007_15385_amd import build as B

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
PACKED = re.compile(r"\bv_pk_(fma|mul|add)_f32\b")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def _kernel_sources():
    return [os.path.basename(p) for p in B.sources() if "__global__" in open(p).read()]


@pytest.mark.parametrize("src", _kernel_sources())
def test_no_packed_fp32_in_device_code(src, tmp_path):
    flags = [f for f in B.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    out = tmp_path / (src + ".s")
    cmd = [HIPCC, *flags, "--cuda-device-only", "-S", "-I", B.INCLUDE, "-I", B.CSRC, "-o", str(out),
           os.path.join(B.CSRC, src)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    asm = out.read_text()
    assert ".amdhsa_kernel" in asm  # the kernels were compiled
    hits = sorted(set(m.group(0) for m in PACKED.finditer(asm)))
    assert not hits, f"{src}: packed float32 instructions {hits}"

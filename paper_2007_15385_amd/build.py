"""Compile the HIP library for gfx950 into the package directory.

    python -m paper_2007_15385_amd.build

builds ``libpip_voronoi.so`` next to this file from ``csrc/*.hip`` with
hipcc: every source is compiled to an object file of its own (in parallel)
and the objects are linked into the shared library.  binary64 code must not
contract multiply-adds (labels and generators are bit-exact replays of the
plain algorithms), so the whole library is compiled with
``-ffp-contract=off``; float32 multiply-adds are explicit ``fmaf`` calls.
Packed float32 instructions are disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libpip_voronoi.so")
ARCH = os.environ.get("PIP_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-ffp-contract=off",
    "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-core results in ordinary VGPRs (the reductions read them directly)
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wall",
    "-Wno-unused-result",
]


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _run(cmd: list[str]) -> subprocess.CompletedProcess:
    return subprocess.run(cmd, capture_output=True, text=True)


def build(verbose: bool = False, extra: list[str] | None = None, out: str = LIB) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    jobs = max(1, min(len(sources()), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with tempfile.TemporaryDirectory(prefix="pipbuild") as tmp:
        cmds = []
        objs = []
        for src in sources():
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            objs.append(obj)
            cmds.append([hipcc, *HIPCC_FLAGS, *(extra or []), "-I", INCLUDE, "-I", CSRC, "-c",
                         "-o", obj, src])
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        with cf.ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(_run, cmds))
        for c, r in zip(cmds, results):
            if r.returncode != 0:
                raise RuntimeError(f"hipcc failed ({r.returncode}) on {c[-1]}:\n{r.stderr[-8000:]}")
            if verbose and r.stderr.strip():
                print(r.stderr[-4000:], file=sys.stderr)
        link = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out + ".tmp", *objs]
        if verbose:
            print(" ".join(link), flush=True)
        r = _run(link)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc link failed ({r.returncode}):\n{r.stderr[-8000:]}")
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))

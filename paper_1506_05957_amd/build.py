"""Build libfmmbem.so (HIP for gfx950) in-tree.

Every source is compiled by hipcc for gfx950 only.  The octree, list and
near-field sources are compiled without floating-point contraction so that
their decisions are reproducible bit for bit; packed FP32 instructions are
disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfmmbem.so")
ARCH = "gfx950"

SOURCES = [
    ("rules.cpp", []),
    ("rotations.cpp", []),
    ("tree.hip", ["-ffp-contract=off"]),
    ("near.hip", ["-ffp-contract=off"]),
    ("translations.hip", []),
    # MFMA accumulators in VGPRs: without it the compiler copies them
    # through AGPRs around every product of the M2L loops
    ("fmm.hip", ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]),
    ("nearfield.hip", []),
    ("krylov.hip", []),
    ("api.hip", []),
    ("server.cpp", []),
]

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    "-Wno-unknown-warning-option", "-Wno-pass-failed",
]


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return p


def _compile(src: str, extra: list[str]) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + extra
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    noise = "'-packed-fp32-ops' is not a recognized feature"
    msg = "\n".join(l for l in r.stderr.splitlines() if noise not in l and l.strip())
    if msg:
        sys.stderr.write(msg + "\n")
    return obj


def build(jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, len(SOURCES))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(*s), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())

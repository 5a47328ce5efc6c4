"""Build libskgemm.so for gfx950 in-tree with hipcc.

Each translation unit under csrc/ is compiled in its own hipcc process (the
kernel instantiations are split per input type so they build in parallel),
then linked into paper_2212_08964_amd/libskgemm.so.
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libskgemm.so")
BUILD_DIR = os.path.join(PKG, "_build")

# the largest units first, so the pool finishes together
SOURCES = ["kernels_bf16.hip", "kernels_bf16_full.hip", "kernels_f16.hip", "kernels_f16_full.hip",
           "kernels_f64.hip", "kernels_f64_full.hip", "kernels_f8.hip", "kernels_f8_full.hip",
           "kernels_f32.hip", "kernels_f32_full.hip", "dispatch.hip", "quant.hip", "noalloc.hip", "pack.hip",
           "skgemm_abi.cpp"]

ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def common_flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            # packed FP32 instructions are kept out of all device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-function"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    cmd = [hipcc(), *common_flags(), "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    elif src.startswith("kernels_"):
        cmd.append("-Rpass-analysis=kernel-resource-usage")
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{res.stderr}")
    if src.startswith("kernels_"):
        check_no_scratch(src, res.stderr)
    return obj


def check_no_scratch(src: str, remarks: str) -> None:
    """Fail the build if a GEMM kernel spills to scratch memory.

    On MI355X a kernel that uses scratch pays a fixed cost of about 20 us per
    launch (measured with two otherwise identical trivial kernels), more than
    the whole runtime of a small GEMM, so a spill is a build error here."""
    name = None
    bad = []
    for line in remarks.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and int(m.group(1)) > 0:
            bad.append(f"{name}: {m.group(1)} bytes/lane")
    if bad:
        raise RuntimeError(f"{src}: kernels use scratch memory:\n  " + "\n  ".join(bad))


def build(verbose: bool = True) -> str:
    """Compile every HIP unit for gfx950 and link libskgemm.so (always rebuilds)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = min(len(SOURCES), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()

"""Compile the gfx950 library ``libkx.so`` in-tree with hipcc.

Usage: ``python -m paper_2411_02640_amd.build`` (also called by
``__graft_entry__.build()`` at the repository root).  Every translation unit is compiled for gfx950 only,
with packed-FP32 instruction selection disabled, then linked into one shared
library next to this file; ``kx_micro.hip`` (elementary-function throughput
probes for the roofline prices) goes into ``libkx_micro.so`` beside it.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libkx.so")
SOURCES = ["kx_api.cpp", "kx_mech.cpp", "kx_serve.cpp", "kx_rates.hip", "kx_transport.hip",
           "kx_jacobian.hip", "kx_qss.hip", "kx_batch.hip"]
MICRO_SOURCE = "kx_micro.hip"
MICRO_LIB = os.path.join(HERE, "libkx_micro.so")
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def common_flags():
    # -amdgpu-mfma-vgpr-form: MFMA accumulators stay in ordinary VGPRs (the
    # accumulation registers would otherwise be copied to and from VGPRs in
    # every iteration of the transport K-loop)
    return ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-mllvm", "-amdgpu-mfma-vgpr-form",
            "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-result"]


def build(verbose: bool = False, jobs: int = 4, tsan: bool = False) -> str:
    """Compile and link libkx.so (and libkx_micro.so).  tsan=True instead
    builds the library with ThreadSanitizer instrumentation of the host code
    only (the GPU code is compiled as usual) into _build/tsan/libkx.so, for
    running the request server's host tests under the sanitizer: load it with
    KX_LIBRARY=<that path> and the clang TSan runtime preloaded."""
    cc = hipcc()
    out_dir = os.path.join(HERE, "_build", "tsan" if tsan else "")
    lib_out = os.path.join(out_dir, "libkx.so") if tsan else LIB
    extra = ["-Xarch_host", "-fsanitize=thread", "-g"] if tsan else []
    os.makedirs(out_dir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(out_dir, src + ".o")
        cmd = [cc, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + common_flags() + extra
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = lib_out + ".tmp"
    cmd = [cc, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib_out)
    if tsan:
        return lib_out
    # the elementary-function throughput probes (a measuring tool the
    # benchmark loads; not part of libkx.so)
    obj = compile_one(MICRO_SOURCE)
    tmp = MICRO_LIB + ".tmp"
    cmd = [cc, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, MICRO_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, tsan="--tsan" in sys.argv))

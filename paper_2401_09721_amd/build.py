"""Build libfgbd.so in-tree with hipcc for gfx950.

Usage: ``python -m paper_2401_09721_amd.build`` (also called by the repository's
build entry point).  Every source is compiled on every call.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libfgbd.so")

SOURCES = ["fgbd_api.hip", "fgbd_sort.hip", "fgbd_graph.hip", "fgbd_noise.hip", "fgbd_filter.hip", "fgbd_poly.hip", "fgbd_io.hip"]

ARCH = "gfx950"
HIPFLAGS = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-core accumulators in ordinary VGPRs: otherwise the compiler keeps
    # loop-carried accumulators in VGPRs and copies them to and from AGPRs
    # around every MFMA, which serialises the loop on each result
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-variable",
    f"-I{INCLUDE}",
    f"-I{CSRC}",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libfgbd)")


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every HIP source for gfx950 and link libfgbd.so next to this file.
    Returns the library path."""
    cc = hipcc()
    tmp = tempfile.mkdtemp(prefix="fgbd_build_")
    try:
        objs = []
        procs = []
        for src in SOURCES:
            obj = os.path.join(tmp, src.replace(".hip", ".o"))
            cmd = [cc, *HIPFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            objs.append(obj)
            if len([p for p in procs if p[2].poll() is None]) >= jobs:
                procs[0][2].wait()
        for src, cmd, p in procs:
            out, _ = p.communicate()
            text = out.decode(errors="replace")
            warn = "\n".join(ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip())
            if p.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n{text}")
            if verbose and warn:
                print(warn)
        tmp_lib = os.path.join(tmp, "libfgbd.so")
        cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp_lib]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
        shutil.move(tmp_lib, LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Build the HIP library libhfmm.so in place (gfx950).

Usage: python -m paper_1703_09136_amd.build

Each source is compiled to an object of its own (in parallel), then linked.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhfmm.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ["hfmm.hip", "kernels.hip", "p2p.hip", "batch.hip", "blocked.hip", "noalloc.hip", "tree.hip", "tree_host.cpp", "tree_api.hip", "bie.hip", "transmit.hip"]
ARCH = os.environ.get("HFMM_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # packed FP32 instructions stay off: some of their forms have
         # given intermittently wrong results on gfx950
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # MFMA accumulators in ordinary VGPRs: with AGPRs the compiler
         # copies every accumulator across on each step of the
         # translation kernel's first contraction loop
         "-mllvm", "-amdgpu-mfma-vgpr-form",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _compile(src: str) -> tuple[str, subprocess.CompletedProcess]:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + FLAGS + ["-c", "-o", obj, os.path.join(CSRC, src)]
    return obj, subprocess.run(cmd, capture_output=True, text=True)


def _report(res, verbose):
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed with status %d" % res.returncode)
    if verbose and res.stderr.strip():
        lines = [ln for ln in res.stderr.splitlines() if "packed-fp32-ops" not in ln]
        if lines:
            sys.stderr.write("\n".join(lines[:40]) + "\n")


def build(verbose: bool = True) -> str:
    """Compile every source and link one shared library; returns its path."""
    os.makedirs(OBJDIR, exist_ok=True)
    sources = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    if verbose:
        print(" ".join([hipcc()] + FLAGS + ["-c"]) + " " + " ".join(sources), flush=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(sources), 8)) as ex:
        results = list(ex.map(_compile, sources))
    objs = []
    for obj, res in results:
        _report(res, verbose)
        objs.append(obj)
    tmp = LIB + ".tmp"
    res = subprocess.run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs,
                         capture_output=True, text=True)
    _report(res, verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())

"""Build the gfx950 shared library libcontentarea.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT_DIR = os.path.join(PKG, "_lib")
LIB_PATH = os.path.join(OUT_DIR, "libcontentarea.so")
SOURCES = ["ca_api.cpp", "ca_server.cpp", "ca_kernels.hip", "ca_ingest.hip", "ca_cnn.hip",
           "ca_cnn2d.hip", "ca_noalloc.hip"]
# the device renderer of synthetic frames: an input generator, built apart
SYNTH_LIB_PATH = os.path.join(OUT_DIR, "libcasynth.so")
SYNTH_SOURCES = ["synth_gpu.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # the numeric contract needs IEEE float/double without fused multiply-add
    "-ffp-contract=off",
    "-fno-fast-math",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA accumulators in architectural VGPRs rather than AGPRs where the
    # budget allows: the 2-D scorer's epilogues then read them without a
    # v_accvgpr_read per element (measured 304-308 -> 292-295 us per 64 x
    # 1080p launch of k_cnn2d_strips, candidates identical)
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wall",
    "-Wno-unused-command-line-argument",
]


def _link(sources, path, verbose):
    tmp = path + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", INCLUDE, *[os.path.join(CSRC, s) for s in sources], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed to build {os.path.basename(path)}")
    os.replace(tmp, path)


def build(verbose: bool = False) -> str:
    """Compile libcontentarea.so and libcasynth.so; returns the former's path."""
    os.makedirs(OUT_DIR, exist_ok=True)
    _link(SOURCES, LIB_PATH, verbose)
    _link(SYNTH_SOURCES, SYNTH_LIB_PATH, verbose)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))

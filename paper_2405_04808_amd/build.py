"""Build libpitmg.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2405_04808_amd.build
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpitmg.so")
SOURCES = ["pitmg_kernels.hip", "pitmg_factor.hip", "pitmg_jacobi_tiled.hip",
           "pitmg_coarse.hip", "pitmg_small.hip", "pitmg_split.hip", "pitmg_gs.hip", "pitmg_unlifted.hip",
           "pitmg_net.hip", "pitmg_host.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off in every HIP translation unit
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]
LINK_FLAGS = []


def hipcc_path() -> str:
    cand = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(cand):
        raise RuntimeError("hipcc not found; the HIP library cannot be built")
    return cand


def build_library(verbose: bool = False) -> str:
    """Compile every HIP source into paper_2405_04808_amd/libpitmg.so."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc_path()] + HIPCC_FLAGS + ["-o", tmp] + srcs + LINK_FLAGS
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libpitmg.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))

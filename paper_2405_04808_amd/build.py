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
           "pitmg_coarse.hip", "pitmg_small.hip", "pitmg_split.hip", "pitmg_gs.hip",
           "pitmg_unlifted.hip", "pitmg_dogleg.hip", "pitmg_net.hip", "pitmg_host.hip"]

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


# Host-side sanitizer build: the same sources with AddressSanitizer and UBSan
# on the host compilation only (each -fsanitize behind -Xarch_host; the GPU
# code is built as usual).  For the CPU checks of the C ABI's validation and
# error paths (tests/test_host_sanitizer.py), never loaded by the package.
SAN_DIR = os.path.join(HERE, "_build")
SAN_LIB = os.path.join(SAN_DIR, "libpitmg_san.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def build_sanitized(verbose: bool = False) -> str:
    """libpitmg_san.so in paper_2405_04808_amd/_build (rebuilt when a source
    is newer)."""
    os.makedirs(SAN_DIR, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    deps = srcs + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    deps.append(os.path.join(HERE, "..", "include", "pitmg.h"))
    if os.path.exists(SAN_LIB) and os.path.getmtime(SAN_LIB) >= max(map(os.path.getmtime, deps)):
        return SAN_LIB
    flags = [f for f in HIPCC_FLAGS if f != "-O3"] + ["-O1"] + SAN_FLAGS
    tmp = SAN_LIB + ".tmp"
    cmd = [hipcc_path()] + flags + ["-o", tmp] + srcs + LINK_FLAGS
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building the sanitized library")
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    print(build_library(verbose=True))

"""The C ABI's host code under AddressSanitizer and UBSan, on the CPU: a
sanitized build of the library (host compilation only) and a small driver
(tests/host_sanitizer_driver.cpp, itself built with both sanitizers) that
exercises option and problem validation, every entry point's NULL-handle
path, the status strings and a setup that fails at its first device call.
Any host memory error or undefined behaviour aborts the driver."""
import os
import shutil
import subprocess

import pytest

from paper_2405_04808_amd import build

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.timeout(900)
def test_abi_host_paths_under_asan_and_ubsan():
    if not (shutil.which("hipcc") or os.path.exists("/opt/rocm/bin/hipcc")):
        pytest.skip("hipcc is not available")
    # the driver links the same sanitizer runtime as the library's host code
    # (the ROCm clang's), not the system compiler's
    gxx = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(gxx):
        pytest.skip("the ROCm clang++ is not available")
    lib = build.build_sanitized()
    exe = os.path.join(build.SAN_DIR, "host_sanitizer_driver")
    src = os.path.join(HERE, "host_sanitizer_driver.cpp")
    res = subprocess.run([gxx, "-std=c++17", "-g", "-O1", "-fsanitize=address",
                          "-fsanitize=undefined", "-fno-omit-frame-pointer", src, "-o", exe,
                          lib, "-Wl,-rpath," + build.SAN_DIR], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    env = dict(os.environ)
    # the HIP runtime keeps process-lifetime allocations; leaks are not checked
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = run.stdout + run.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert "runtime error" not in out, out[-4000:]
    assert run.returncode == 0, out[-4000:]
    assert "0 failure(s)" in run.stdout

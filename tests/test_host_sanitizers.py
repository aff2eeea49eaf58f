"""The host code of the library (model tables, the Formula (5) solver, the
model constructor and every argument check of the C ABI that runs without a
device) built with AddressSanitizer, LeakSanitizer and UndefinedBehaviorSanitizer
and exercised on valid and invalid input by the checks in tests/sanitize/abi_checks.cpp.
The device code is not part of this build: tests/sanitize/launcher_stubs.cpp
stands in for the kernel launchers, which no call reaches without a GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1303_4624_amd", "csrc")
ROCM = "/opt/rocm"


def test_host_code_under_address_and_ub_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists(os.path.join(ROCM, "lib", "libamdhip64.so")):
        pytest.skip("needs g++ and the HIP runtime library")
    exe = str(tmp_path / "abi_checks")
    srcs = [os.path.join(CSRC, "lbm_api.cpp"), os.path.join(CSRC, "lbm_model_host.cpp"),
            os.path.join(ROOT, "tests", "sanitize", "abi_checks.cpp"),
            os.path.join(ROOT, "tests", "sanitize", "launcher_stubs.cpp")]
    cmd = [gxx, "-std=c++20", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, *srcs,
           "-L", os.path.join(ROCM, "lib"), f"-Wl,-rpath,{ROCM}/lib", "-lamdhip64", "-lquadmath",
           "-o", exe]
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                         timeout=600)
    assert res.returncode == 0, res.stdout[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                         timeout=300, env=env, cwd=str(tmp_path))
    assert run.returncode == 0 and run.stdout.strip().endswith("ok"), run.stdout[-4000:]

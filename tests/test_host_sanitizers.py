"""The library's host layer under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

vtx_host.cpp is compiled with g++ (host code only, no device code) together with
tests/sanitize_driver.cpp, which drives every host path that runs without a GPU (Gauss rules,
angular-weight tables, option defaults, every entry point's argument checks, the device check)
and stubs the kernel launchers. Any sanitizer report aborts the run (-fno-sanitize-recover);
leak detection is on.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = "/opt/rocm"


def test_host_layer_under_asan_ubsan(tmp_path):
    gxx = shutil.which("g++")
    if not gxx or not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime.h")):
        pytest.skip("g++ or the HIP headers not available")
    exe = tmp_path / "vtx_san"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include",
           os.path.join(ROOT, "tests", "sanitize_driver.cpp"),
           os.path.join(ROOT, "paper_1404_1719_amd", "csrc", "vtx_host.cpp"),
           f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib", "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               HIP_VISIBLE_DEVICES="", ROCR_VISIBLE_DEVICES="")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host layer ok, 0 failures" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr

"""The library's host code (geometry and coefficient tables, orbit builders,
the binomial checkpoint schedule) built with the host compiler under the
address and undefined-behaviour sanitizers and run over many inputs,
including edge cases and invalid ones (tests/host_sanitize_check.cpp).
Device code is not built here."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1001_3631_amd", "csrc")
ROCM_INC = "/opt/rocm/include"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(ROCM_INC),
                    reason="needs a host C++ compiler and the HIP headers")
def test_host_code_under_address_and_ub_sanitizers(tmp_path):
    exe = tmp_path / "host_sanitize_check"
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-D__HIP_PLATFORM_AMD__", "-I", ROCM_INC, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(HERE, "host_sanitize_check.cpp"),
           os.path.join(CSRC, "geometry.cpp"), os.path.join(CSRC, "orbit.cpp"), os.path.join(CSRC, "revolve.cpp"),
           "-o", str(exe)]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    print(out.stdout[-4000:], out.stderr[-4000:])
    assert out.returncode == 0 and "host checks: 0 failed" in out.stdout

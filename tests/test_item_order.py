"""The streaming kernels' dispatch order (csrc/item_order.h), checked on the
host: built with the host compiler (with address and undefined-behaviour
sanitizers) and run over many grid shapes; see tests/item_order_check.cpp."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1001_3631_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_dispatch_order_is_a_bijection_onto_the_items(tmp_path):
    exe = tmp_path / "item_order_check"
    subprocess.run(["g++", "-O1", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", CSRC, os.path.join(HERE, "item_order_check.cpp"), "-o", str(exe)], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0")
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=env)
    print(out.stdout, out.stderr)
    assert out.returncode == 0 and "bad 0" in out.stdout

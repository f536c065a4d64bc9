"""The host operator build under the address and undefined-behaviour
sanitizers: tests/sanitize_host_build.cpp (constant, x-dependent, x,v-dependent
and v-dependent general coefficient sets at orders 1 to 3, the rejected
forms and degenerate grids) is compiled with paper_2207_09776_amd/csrc/
ops_build.cpp by g++ for the host only and run; a sanitizer report or an
unexpected build status fails the test."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2207_09776_amd", "csrc")
ROCM_INC = "/opt/rocm/include"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(ROCM_INC),
                    reason="needs g++ and the ROCm headers")
def test_operator_build_is_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "sanitize_host_build")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-D__HIP_PLATFORM_AMD__", "-I", ROCM_INC, "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, os.path.join(HERE, "sanitize_host_build.cpp"), "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stderr[-4000:]
    # verify_asan_link_order=0: the environment may preload other libraries
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    out = run.stdout + run.stderr
    assert run.returncode == 0, out[-6000:]
    assert out.rstrip().endswith("ok") or "\nok\n" in out, out[-6000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-6000:]

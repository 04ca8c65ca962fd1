"""Host-side serving logic under the sanitizers: the scratch pool and the FIFO admission of the
serving loop (paper_2206_01382_amd/csrc/server_pool.hpp, which has no HIP dependency) are built
for the CPU with AddressSanitizer and UndefinedBehaviorSanitizer and driven through randomised
request streams (tests/host/pool_admission_check.cpp)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_pool_and_admission_under_asan_ubsan(tmp_path):
    exe = tmp_path / "pool_admission_check"
    src = os.path.join(HERE, "host", "pool_admission_check.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-static-libasan", src, "-o", str(exe)],
                   check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "passed" in r.stdout

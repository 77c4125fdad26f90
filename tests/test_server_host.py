"""The serving loop's host logic (gk_server.hip compiled as host C++) on the
CPU, against the stand-in HIP runtime and kernels of tests/server_check.cpp:
admission, parts spread over ticks, copy-back offsets, the sequential mode,
cancellation and injected failures, plain and under the address /
undefined-behaviour and thread sanitizers.  No GPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2103_14978_amd", "csrc")
# clang: the thread sanitizer of g++ 11 does not intercept
# pthread_cond_clockwait (behind condition_variable::wait_for) and reports the
# waiting thread as still holding its mutex
CXX = "/opt/rocm/llvm/bin/clang++" if os.path.exists("/opt/rocm/llvm/bin/clang++") else None
ROCM_INCLUDE = "/opt/rocm/include"
ROCM_LIB = "/opt/rocm/lib"        # trace ranges (roctx)


@pytest.mark.skipif(CXX is None or not os.path.isdir(ROCM_INCLUDE),
                    reason="clang++ or the HIP headers not found")
@pytest.mark.parametrize("sanitize", [None, "address,undefined", "thread"])
def test_server_host_logic(tmp_path, sanitize):
    exe = tmp_path / "server_check"
    cmd = [CXX, "-std=c++17", "-O1", "-g", "-pthread", "-D__HIP_PLATFORM_AMD__",
           "-I", ROCM_INCLUDE, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-x", "c++", os.path.join(CSRC, "gk_server.hip"),
           "-x", "c++", os.path.join(HERE, "server_check.cpp"),
           os.path.join(CSRC, "gk_host_encode.cpp"), "-L", ROCM_LIB,
           "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{ROCM_LIB}", "-o", str(exe)]
    if sanitize:
        cmd[5:5] = [f"-fsanitize={sanitize}", "-fno-sanitize-recover=all"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "server check ok" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr

"""The host-to-host pipeline's host logic (gk_host.hip compiled as host C++)
on the CPU, against the stand-in HIP runtime of tests/standin_hip.h and the
stand-in kernels of tests/host_check.cpp: the ring of three device slots,
the three streams and their events under random delays, read chunks shared
by pair chunks, the device-memory bound and the offset checks, plain and
under the address / undefined-behaviour and thread sanitizers.  No GPU."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2103_14978_amd", "csrc")
# clang: the thread sanitizer of g++ 11 does not intercept
# pthread_cond_clockwait (behind condition_variable::wait_for)
CXX = "/opt/rocm/llvm/bin/clang++" if os.path.exists("/opt/rocm/llvm/bin/clang++") else None
ROCM_INCLUDE = "/opt/rocm/include"
ROCM_LIB = "/opt/rocm/lib"        # trace ranges (roctx)


@pytest.mark.skipif(CXX is None or not os.path.isdir(ROCM_INCLUDE),
                    reason="clang++ or the HIP headers not found")
@pytest.mark.parametrize("sanitize", [None, "address,undefined", "thread"])
def test_host_pipe_logic(tmp_path, sanitize):
    exe = tmp_path / "host_check"
    cmd = [CXX, "-std=c++17", "-O1", "-g", "-pthread", "-D__HIP_PLATFORM_AMD__",
           "-I", ROCM_INCLUDE, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-x", "c++", os.path.join(CSRC, "gk_host.hip"),
           "-x", "c++", os.path.join(HERE, "host_check.cpp"),
           os.path.join(CSRC, "gk_host_encode.cpp"), "-L", ROCM_LIB,
           "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{ROCM_LIB}", "-o", str(exe)]
    if sanitize:
        cmd[5:5] = [f"-fsanitize={sanitize}", "-fno-sanitize-recover=all"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "host pipe check ok" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr

"""Host code under sanitizers, on the CPU: the read encoder of gk_filter_host
and its worker pool, built from the library's own source with the address +
undefined-behaviour sanitizers and, separately, the thread sanitizer, then
run by tests/host_encode_check.cpp.  No GPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2103_14978_amd", "csrc")
CXX = shutil.which("g++")


@pytest.mark.skipif(CXX is None, reason="g++ not found")
@pytest.mark.parametrize("sanitize", ["address,undefined", "thread"])
def test_host_encoder_under_sanitizer(tmp_path, sanitize):
    exe = tmp_path / "host_encode_check"
    cmd = [CXX, "-std=c++17", "-O1", "-g", "-pthread", f"-fsanitize={sanitize}",
           "-fno-sanitize-recover=all", "-I", CSRC,
           os.path.join(HERE, "host_encode_check.cpp"), os.path.join(CSRC, "gk_host_encode.cpp"),
           "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert "host encode check ok" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr

"""The served bench's native load generator (gk_loadgen.cpp) on the CPU,
against a stand-in server (tests/loadgen_check.cpp), plain and under the
address / undefined-behaviour and thread sanitizers.  No GPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2103_14978_amd", "csrc")
CXX = shutil.which("g++")


@pytest.mark.skipif(CXX is None, reason="g++ not found")
@pytest.mark.parametrize("sanitize", [None, "address,undefined", "thread"])
def test_loadgen_against_stand_in_server(tmp_path, sanitize):
    exe = tmp_path / "loadgen_check"
    cmd = [CXX, "-std=c++17", "-O1", "-g", "-pthread", "-I", os.path.join(ROOT, "include"),
           os.path.join(HERE, "loadgen_check.cpp"), os.path.join(CSRC, "gk_loadgen.cpp"),
           "-o", str(exe)]
    if sanitize:
        cmd[3:3] = [f"-fsanitize={sanitize}", "-fno-sanitize-recover=all"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert "loadgen check ok" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr

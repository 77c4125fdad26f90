"""The binding's ctypes structures have the header's layout: a C probe
compiled against include/gk.h prints every field offset and struct size, and
the ctypes classes must agree (CPU only; gcc)."""
import os
import subprocess

import pytest

from conftest import ROOT

STRUCTS = {
    "gk_batch": ["n_reads", "pitch", "max_read_len", "e_uniform", "read_layout", "reads",
                 "read_len", "read_has_n", "n_pairs", "pair_read", "cand_pos", "e", "accept",
                 "est", "accept_bits", "flags"],
    "gk_host_batch": ["n_reads", "max_read_len", "ascii", "read_off", "n_pairs", "pair_read",
                      "cand_pos", "e", "e_uniform", "accept", "est", "flags", "packed",
                      "read_len", "read_has_n", "packed_layout"],
    "gk_request": ["reads", "read_off", "n_reads", "e", "pair_read", "cand_pos", "n_pairs",
                   "accept", "est", "t_arrival_us"],
    "gk_request_stats": ["status", "n_pairs", "t_submit_us", "t_admit_us", "t_done_us"],
    "gk_tick_record": ["t_launch_us", "t_kernel_done_us", "t_done_us", "n_requests",
                       "reserved", "n_pairs"],
}


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    d = tmp_path_factory.mktemp("abi")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "gk.h"', "int main(void) {"]
    for name, fields in STRUCTS.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f in fields:
            lines.append(f'printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["return 0;", "}"]
    src = d / "probe.c"
    src.write_text("\n".join(lines))
    exe = d / "probe"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        s, f, v = line.split()
        got[(s, f)] = int(v)
    return got


@pytest.mark.parametrize("name", list(STRUCTS))
def test_struct_layout_matches_header(c_layout, name):
    import ctypes
    from paper_2103_14978_amd import gk
    cls = getattr(gk, name)
    assert [f for f, _ in cls._fields_] == STRUCTS[name]
    assert ctypes.sizeof(cls) == c_layout[(name, "size")]
    for f in STRUCTS[name]:
        assert getattr(cls, f).offset == c_layout[(name, f)], f"{name}.{f}"


def test_constants_match_header():
    import re
    from paper_2103_14978_amd import gk
    hdr = open(os.path.join(ROOT, "include", "gk.h")).read()
    for name in ("GK_FLAG_NO_REFINE", "GK_FLAG_HAMMING_FASTPATH", "GK_VERIFY_MAX_E",
                 "GK_MAX_READ_LEN", "GK_READS_SPLIT", "GK_READS_INTERLEAVED",
                 "GK_NOALLOC_MAX_PAIRS"):
        m = re.search(rf"#define\s+{name}\s+(\w+)", hdr)
        assert m, name
        assert int(m.group(1).rstrip("uU").rstrip("uU"), 0) == getattr(gk, name), name


def test_readme_c_example_compiles(tmp_path):
    """The C example in README.md compiles against include/gk.h."""
    import re
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    text = open(os.path.join(root, "README.md")).read()
    blocks = re.findall(r"```c\n(.*?)```", text, re.S)
    assert blocks, "no C example in README.md"
    src = tmp_path / "example.c"
    src.write_text(blocks[0])
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-I",
                        os.path.join(root, "include"), "-c", str(src), "-o",
                        str(tmp_path / "example.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr

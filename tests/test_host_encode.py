"""The host-side read encoder of gk_filter_host (GK_OPT_HOST_ENCODE_THREADS)
against the encoding rule written out here: A/C/G/T (either case) -> 0..3
(Sec. 2.1), 16 bases per word with the low code bits in bits 0-15 and the
high code bits in bits 16-31; any other byte takes the GPU encoder's code
((c >> 1) ^ (c >> 2)) & 3 and marks the read as holding an unknown base; only
the first 16 * rows bytes of a read are encoded; lengths are capped at 65535.
Host code only: runs without a GPU."""
import ctypes

import numpy as np
import pytest

from paper_2103_14978_amd import gk

_TABLE = {ord(ch): code for code, ch in enumerate("ACGT")}
_TABLE.update({ord(ch): code for code, ch in enumerate("acgt")})


def expected(text: bytes, off: np.ndarray, rows: int):
    n = len(off) - 1
    words = np.zeros((n, rows), np.uint32)
    lens = np.zeros(n, np.uint16)
    has_n = np.zeros(n, np.uint8)
    for r in range(n):
        read = text[off[r]:off[r + 1]]
        lens[r] = min(len(read), 0xFFFF)
        for i, c in enumerate(read[:16 * rows]):
            if c in _TABLE:
                code = _TABLE[c]
            else:
                code = ((c >> 1) ^ (c >> 2)) & 3
                has_n[r] = 1
            w, j = divmod(i, 16)
            words[r, w] |= ((code & 1) << j) | ((code >> 1) << (16 + j))
    return words.reshape(-1), lens, has_n


def encode(text: bytes, off: np.ndarray, rows: int, sse2_only: bool):
    """The library's encoder; sse2_only forces the path for CPUs without
    AVX2 (the default path takes AVX2 where the CPU has it)."""
    lib = gk.lib()
    fn = lib.gk_detail_host_encode_rows
    fn.restype = None
    fn.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    n = len(off) - 1
    buf = np.frombuffer(text, np.uint8).copy() if text else np.zeros(0, np.uint8)
    off = np.ascontiguousarray(off, np.uint64)
    words = np.full(n * rows, 0xDEADBEEF, np.uint32)
    lens = np.full(n, 0xABCD, np.uint16)
    has_n = np.full(n, 7, np.uint8)
    fn(buf.ctypes.data, off.ctypes.data, n, rows, words.ctypes.data, lens.ctypes.data,
       has_n.ctypes.data, int(sse2_only))
    return words, lens, has_n


@pytest.mark.parametrize("sse2_only", [False, True], ids=["default", "sse2"])
@pytest.mark.parametrize("rows", [1, 4, 7, 32])
def test_host_encoder_matches_rule(rows, sse2_only):
    rng = np.random.default_rng(100 + rows)
    alphabet = np.frombuffer(b"ACGTACGTACGTacgtNnX-.", np.uint8)
    lens = rng.integers(0, 16 * rows + 40, 400)
    lens[:6] = [0, 1, 15, 16, 17, 16 * rows]
    parts = []
    for k, m in enumerate(lens):
        pool = alphabet if k % 3 == 0 else alphabet[:12]
        parts.append(pool[rng.integers(0, len(pool), int(m))].tobytes())
    text = b"".join(parts)
    off = np.zeros(len(parts) + 1, np.uint64)
    np.cumsum([len(p) for p in parts], out=off[1:])
    got = encode(text, off, rows, sse2_only)
    want = expected(text, off.astype(np.int64), rows)
    for g, w, what in zip(got, want, ("words", "lengths", "unknown flags")):
        assert np.array_equal(g, w), what


@pytest.mark.parametrize("sse2_only", [False, True], ids=["default", "sse2"])
def test_host_encoder_long_and_edge_reads(sse2_only):
    """A read longer than 65535 bases (length capped), a read ending exactly
    at the end of the text with a partial last word, and empty reads."""
    rng = np.random.default_rng(7)
    acgt = np.frombuffer(b"ACGT", np.uint8)
    parts = [b"", acgt[rng.integers(0, 4, 70000)].tobytes(), b"",
             acgt[rng.integers(0, 4, 37)].tobytes()]
    text = b"".join(parts)
    off = np.zeros(len(parts) + 1, np.uint64)
    np.cumsum([len(p) for p in parts], out=off[1:])
    got = encode(text, off, 32, sse2_only)
    want = expected(text, off.astype(np.int64), 32)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    assert got[1][1] == 0xFFFF and got[1][3] == 37

"""GateKeeper-GPU oracle: ctypes binding to the plain per-base C oracle.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package; the product library
never links or calls it, and it shares no code with the HIP path.

The C source (``gk_oracle.c``) restates the filter of GateKeeper-GPU
(Sec. 2.1 for the GateKeeper steps, Sec. 3.3 for unknown bases, Sec. 3.4 for
the leading/trailing refinement) one base at a time on ASCII strings.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gk_oracle.c")
LIB = os.path.join(HERE, "libgk_oracle.so")

REJECT, ACCEPT, UNDEFINED, INVALID = 0, 1, 2, 3
EST_NONE = 0xFFFF
MAX_LEN = 512
NO_REFINE = 1
HAMMING_FASTPATH = 2
STAGE_RAW, STAGE_AMENDED, STAGE_REFINED = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no SIMD intrinsics)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
             "-pthread", SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ctypes.CDLL(LIB)
        c_char_p, u8p, u16p, u32p, u64p = (ctypes.c_char_p,
                                           ctypes.POINTER(ctypes.c_uint8),
                                           ctypes.POINTER(ctypes.c_uint16),
                                           ctypes.POINTER(ctypes.c_uint32),
                                           ctypes.POINTER(ctypes.c_uint64))
        L.gko_amend.argtypes = [u8p, ctypes.c_uint32, u8p]
        L.gko_amend.restype = ctypes.c_int
        L.gko_filter_pair.argtypes = [c_char_p, ctypes.c_uint32, c_char_p, ctypes.c_uint64,
                                      ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, u16p]
        L.gko_filter_pair.restype = ctypes.c_uint32
        L.gko_filter_pair_trace.argtypes = L.gko_filter_pair.argtypes + [u8p]
        L.gko_filter_pair_trace.restype = ctypes.c_uint32
        L.gko_filter_batch.argtypes = [ctypes.c_void_p, u64p, ctypes.c_uint32, ctypes.c_void_p,
                                       ctypes.c_uint64, u32p, u32p, u8p, ctypes.c_uint32,
                                       ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                       u8p, u16p]
        L.gko_filter_batch.restype = ctypes.c_int
        L.gko_levenshtein.argtypes = [c_char_p, ctypes.c_uint32, c_char_p, ctypes.c_uint32,
                                      ctypes.c_uint32]
        L.gko_levenshtein.restype = ctypes.c_uint32
        L.gko_levenshtein_full.argtypes = [c_char_p, ctypes.c_uint32, c_char_p, ctypes.c_uint32]
        L.gko_levenshtein_full.restype = ctypes.c_uint32
        L.gko_levenshtein_batch.argtypes = [ctypes.c_void_p, u64p, ctypes.c_uint32,
                                            ctypes.c_void_p, ctypes.c_uint64, u32p, u32p,
                                            ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                            u16p]
        L.gko_levenshtein_batch.restype = ctypes.c_int
        _lib = L
    return _lib


def _b(s) -> bytes:
    return s.encode() if isinstance(s, str) else bytes(s)


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def amend(bits) -> list[int]:
    """Amend one 0/1 mask (list or array of ints)."""
    a = np.ascontiguousarray(np.asarray(bits, dtype=np.uint8))
    out = np.empty_like(a)
    lib().gko_amend(_ptr(a, ctypes.c_uint8), len(a), _ptr(out, ctypes.c_uint8))
    return out.tolist()


def filter_pair(read, ref, pos: int, e: int, flags: int = 0) -> tuple[int, int]:
    """(result code, edit estimate) for read against ref[pos, pos+len(read))."""
    r, g = _b(read), _b(ref)
    est = ctypes.c_uint16(0)
    res = lib().gko_filter_pair(r, len(r), g, len(g), pos, e, flags, ctypes.byref(est))
    return int(res), int(est.value)


def filter_trace(read, ref, pos: int, e: int, flags: int = 0):
    """(result, est, masks) where masks[slot][stage] is a list of 0/1.

    Slot 0 is the Hamming mask, slot 2k-1 the deletion mask for shift +k and
    slot 2k the insertion mask for shift -k."""
    r, g = _b(read), _b(ref)
    m = len(r)
    e_eff = min(e, m)
    buf = np.zeros((2 * e_eff + 1) * 3 * max(m, 1), dtype=np.uint8)
    est = ctypes.c_uint16(0)
    res = lib().gko_filter_pair_trace(r, m, g, len(g), pos, e, flags, ctypes.byref(est),
                                      _ptr(buf, ctypes.c_uint8))
    masks = buf.reshape(2 * e_eff + 1, 3, max(m, 1))[:, :, :m].tolist()
    return int(res), int(est.value), masks


def filter_batch(reads: np.ndarray, read_off: np.ndarray, ref: np.ndarray,
                 pair_read: np.ndarray, cand_pos: np.ndarray, e, flags: int = 0,
                 n_threads: int = 1):
    """Filter many pairs.  reads/ref are uint8 ASCII arrays, read_off uint64
    offsets (n_reads + 1), pair_read/cand_pos uint32 per pair, e an int or a
    uint8 array per pair.  Returns (accept uint8, est uint16)."""
    reads = np.ascontiguousarray(reads, dtype=np.uint8)
    read_off = np.ascontiguousarray(read_off, dtype=np.uint64)
    ref = np.ascontiguousarray(ref, dtype=np.uint8)
    pair_read = np.ascontiguousarray(pair_read, dtype=np.uint32)
    cand_pos = np.ascontiguousarray(cand_pos, dtype=np.uint32)
    n = len(cand_pos)
    assert len(pair_read) == n
    accept = np.empty(n, dtype=np.uint8)
    est = np.empty(n, dtype=np.uint16)
    if np.isscalar(e) or isinstance(e, int):
        e_arr, e_u = None, int(e)
    else:
        e_arr = np.ascontiguousarray(e, dtype=np.uint8)
        assert len(e_arr) == n
        e_u = 0
    lib().gko_filter_batch(
        reads.ctypes.data, _ptr(read_off, ctypes.c_uint64), len(read_off) - 1,
        ref.ctypes.data, len(ref), _ptr(pair_read, ctypes.c_uint32),
        _ptr(cand_pos, ctypes.c_uint32),
        _ptr(e_arr, ctypes.c_uint8) if e_arr is not None else None, e_u, n, flags,
        n_threads, _ptr(accept, ctypes.c_uint8), _ptr(est, ctypes.c_uint16))
    return accept, est


def levenshtein(a, b, cap: int | None = None) -> int:
    a, b = _b(a), _b(b)
    if cap is None:
        return int(lib().gko_levenshtein_full(a, len(a), b, len(b)))
    return int(lib().gko_levenshtein(a, len(a), b, len(b), cap))


def levenshtein_batch(reads, read_off, ref, pair_read, cand_pos, cap: int,
                      n_threads: int = 1) -> np.ndarray:
    reads = np.ascontiguousarray(reads, dtype=np.uint8)
    read_off = np.ascontiguousarray(read_off, dtype=np.uint64)
    ref = np.ascontiguousarray(ref, dtype=np.uint8)
    pair_read = np.ascontiguousarray(pair_read, dtype=np.uint32)
    cand_pos = np.ascontiguousarray(cand_pos, dtype=np.uint32)
    n = len(cand_pos)
    out = np.empty(n, dtype=np.uint16)
    lib().gko_levenshtein_batch(
        reads.ctypes.data, _ptr(read_off, ctypes.c_uint64), len(read_off) - 1,
        ref.ctypes.data, len(ref), _ptr(pair_read, ctypes.c_uint32),
        _ptr(cand_pos, ctypes.c_uint32), n, cap, n_threads, _ptr(out, ctypes.c_uint16))
    return out

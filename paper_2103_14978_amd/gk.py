"""Python binding of libgk (include/gk.h): same names, argument marshalling
only.  Device buffers are passed as raw device addresses; torch tensors are
accepted and passed by ``data_ptr()``.  Streams are raw hipStream_t handles
(``torch.cuda.current_stream().cuda_stream``) or torch streams.

Every step of the filter runs in the HIP library.  This module has no
fallback: if libgk.so is missing it raises, it never computes anything
itself.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgk.so")

GK_OK, GK_EINVAL, GK_ENOMEM, GK_EDEVICE, GK_ENOREF, GK_ERANGE = 0, -1, -2, -3, -4, -5
GK_ETIMEOUT = -7
GK_ECANCELED = -8
GK_SERVER_BATCHED, GK_SERVER_SEQUENTIAL = 0, 1
GK_REJECT, GK_ACCEPT, GK_UNDEFINED, GK_INVALID = 0, 1, 2, 3
GK_EST_NONE = 0xFFFF
GK_VERIFY_MAX_E = 31
GK_FLAG_NO_REFINE = 1
GK_FLAG_HAMMING_FASTPATH = 2
GK_MAX_READ_LEN = 512
GK_NOALLOC_MAX_PAIRS = 1 << 22
GK_READS_SPLIT, GK_READS_INTERLEAVED = 0, 1
GK_OPT_PAIRS_PER_LANE = 1
GK_OPT_MIXED_TILE = 2
GK_OPT_MIXED_PAIRS_PER_LANE = 3
GK_OPT_MIXED_SORT_E = 4
GK_OPT_MIXED_BLOCKS_PER_CU = 5
GK_OPT_MIXED_GRAPH = 6
GK_OPT_HOST_ENCODE_THREADS = 7
GK_OPT_SERVER_PART_PAIRS = 8
GK_OPT_SERVER_TICK_PAIRS = 9
GK_OPT_HOST_CHUNK_PAIRS = 10
GK_OPT_SERVER_COPY_STREAMS = 11
STATUS_NAMES = {0: "GK_OK", -1: "GK_EINVAL", -2: "GK_ENOMEM", -3: "GK_EDEVICE",
                -4: "GK_ENOREF", -5: "GK_ERANGE", -7: "GK_ETIMEOUT", -8: "GK_ECANCELED"}


class GkError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class gk_batch(ctypes.Structure):
    _fields_ = [
        ("n_reads", ctypes.c_uint32),
        ("pitch", ctypes.c_uint32),
        ("max_read_len", ctypes.c_uint32),
        ("e_uniform", ctypes.c_uint32),
        ("read_layout", ctypes.c_uint32),
        ("reads", ctypes.c_void_p),
        ("read_len", ctypes.c_void_p),
        ("read_has_n", ctypes.c_void_p),
        ("n_pairs", ctypes.c_uint64),
        ("pair_read", ctypes.c_void_p),
        ("cand_pos", ctypes.c_void_p),
        ("e", ctypes.c_void_p),
        ("accept", ctypes.c_void_p),
        ("est", ctypes.c_void_p),
        ("accept_bits", ctypes.c_void_p),
        ("flags", ctypes.c_uint32),
    ]


class gk_host_batch(ctypes.Structure):
    _fields_ = [
        ("n_reads", ctypes.c_uint32),
        ("max_read_len", ctypes.c_uint32),
        ("ascii", ctypes.c_void_p),
        ("read_off", ctypes.c_void_p),
        ("n_pairs", ctypes.c_uint64),
        ("pair_read", ctypes.c_void_p),
        ("cand_pos", ctypes.c_void_p),
        ("e", ctypes.c_void_p),
        ("e_uniform", ctypes.c_uint32),
        ("accept", ctypes.c_void_p),
        ("est", ctypes.c_void_p),
        ("flags", ctypes.c_uint32),
        ("packed", ctypes.c_void_p),
        ("read_len", ctypes.c_void_p),
        ("read_has_n", ctypes.c_void_p),
        ("packed_layout", ctypes.c_uint32),
    ]


class gk_request(ctypes.Structure):
    _fields_ = [
        ("reads", ctypes.c_void_p),
        ("read_off", ctypes.c_void_p),
        ("n_reads", ctypes.c_uint32),
        ("e", ctypes.c_uint32),
        ("pair_read", ctypes.c_void_p),
        ("cand_pos", ctypes.c_void_p),
        ("n_pairs", ctypes.c_uint64),
        ("accept", ctypes.c_void_p),
        ("est", ctypes.c_void_p),
        ("t_arrival_us", ctypes.c_int64),
    ]


class gk_request_stats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("n_pairs", ctypes.c_uint64),
        ("t_submit_us", ctypes.c_int64),
        ("t_admit_us", ctypes.c_int64),
        ("t_done_us", ctypes.c_int64),
    ]


class gk_tick_record(ctypes.Structure):
    _fields_ = [
        ("t_launch_us", ctypes.c_int64),
        ("t_kernel_done_us", ctypes.c_int64),
        ("t_done_us", ctypes.c_int64),
        ("n_requests", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("n_pairs", ctypes.c_uint64),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libgk.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2103_14978_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        L.gk_create.argtypes = [i32, ctypes.POINTER(vp)]
        L.gk_create.restype = i32
        L.gk_destroy.argtypes = [vp]
        L.gk_destroy.restype = None
        L.gk_last_error.argtypes = [vp]
        L.gk_last_error.restype = ctypes.c_char_p
        L.gk_load_reference.argtypes = [vp, ctypes.c_char_p, u64]
        L.gk_load_reference.restype = i32
        L.gk_load_reference_2bit.argtypes = [vp, vp, u64, u32, vp, u64]
        L.gk_load_reference_2bit.restype = i32
        L.gk_reference_info.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64)]
        L.gk_reference_info.restype = i32
        L.gk_encode_reads.argtypes = [vp, vp, vp, u32, u32, u32, u32, vp, vp, vp, vp]
        L.gk_encode_reads.restype = i32
        L.gk_filter.argtypes = [vp, ctypes.POINTER(gk_batch), vp]
        L.gk_filter.restype = i32
        L.gk_filter_ascii.argtypes = [vp, ctypes.POINTER(gk_batch), vp, vp, vp]
        L.gk_filter_ascii.restype = i32
        L.gk_filter_host.argtypes = [vp, ctypes.POINTER(gk_host_batch)]
        L.gk_filter_host.restype = i32
        L.gk_verify.argtypes = [vp, ctypes.POINTER(gk_batch), vp, vp, vp]
        L.gk_verify.restype = i32
        L.gk_filter_mixed.argtypes = [vp, ctypes.POINTER(gk_batch), vp]
        L.gk_filter_mixed.restype = i32
        L.gk_filter_mixed_noalloc.argtypes = [vp, ctypes.POINTER(gk_batch), vp]
        L.gk_filter_mixed_noalloc.restype = i32
        L.gk_tune_mixed.argtypes = [vp, ctypes.POINTER(gk_batch), vp, u64, ctypes.c_char_p,
                                    ctypes.c_char_p, ctypes.c_size_t]
        L.gk_tune_mixed.restype = i32
        L.gk_server_start.argtypes = [vp, u64, u32, u32, u32, ctypes.POINTER(vp)]
        L.gk_server_start.restype = i32
        L.gk_server_submit.argtypes = [vp, ctypes.POINTER(gk_request), ctypes.POINTER(u64)]
        L.gk_server_submit.restype = i32
        L.gk_server_wait.argtypes = [vp, u64, ctypes.c_int64, ctypes.POINTER(gk_request_stats)]
        L.gk_server_wait.restype = i32
        L.gk_server_counters.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64),
                                         ctypes.POINTER(u64)]
        L.gk_server_counters.restype = i32
        L.gk_server_tick_log.argtypes = [vp, ctypes.POINTER(gk_tick_record), u64,
                                         ctypes.POINTER(u64)]
        L.gk_server_tick_log.restype = i32
        L.gk_server_stop.argtypes = [vp]
        L.gk_server_stop.restype = i32
        L.gk_clock_us.argtypes = []
        L.gk_clock_us.restype = ctypes.c_int64
        L.gk_set_option.argtypes = [vp, i32, ctypes.c_int64]
        L.gk_set_option.restype = i32
        L.gk_get_option.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int64)]
        L.gk_get_option.restype = i32
        _lib = L
    return _lib


EXPORTED = ("gk_create", "gk_destroy", "gk_last_error", "gk_load_reference",
            "gk_load_reference_2bit", "gk_reference_info", "gk_encode_reads", "gk_filter",
            "gk_filter_ascii", "gk_filter_host", "gk_verify", "gk_set_option",
            "gk_get_option", "gk_filter_mixed", "gk_filter_mixed_noalloc", "gk_tune_mixed",
            "gk_server_start", "gk_server_submit", "gk_server_wait", "gk_server_counters",
            "gk_server_tick_log", "gk_server_stop", "gk_clock_us")


def ptr(x) -> int | None:
    """Device address of a torch tensor, an int, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def stream_handle(s) -> int | None:
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return int(s.cuda_stream)


def _check(ctx, status: int, what: str):
    if status != GK_OK:
        msg = lib().gk_last_error(ctx)
        raise GkError(status, f"{what}: {msg.decode() if msg else ''}")


def gk_create(device: int = 0) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    st = lib().gk_create(device, ctypes.byref(h))
    _check(None, st, "gk_create")
    return h


def gk_destroy(ctx) -> None:
    lib().gk_destroy(ctx)


def gk_last_error(ctx) -> str:
    m = lib().gk_last_error(ctx)
    return m.decode() if m else ""


def gk_load_reference(ctx, ascii) -> None:
    """ascii: bytes or a uint8 numpy array in host memory."""
    if not isinstance(ascii, (bytes, bytearray)):
        import numpy as np
        a = np.ascontiguousarray(ascii, dtype=np.uint8)
        buf = ctypes.cast(a.ctypes.data, ctypes.c_char_p)
        n = a.size
        st = lib().gk_load_reference(ctx, buf, n)
    else:
        st = lib().gk_load_reference(ctx, bytes(ascii), len(ascii))
    _check(ctx, st, "gk_load_reference")


def gk_load_reference_2bit(ctx, packed, length: int, layout: int, runs=None) -> None:
    """packed: host uint32 array of ceil(length / 16) words in `layout`;
    runs: host array of (start, length) pairs of unknown bases, or None."""
    import numpy as np
    p = np.ascontiguousarray(packed, dtype=np.uint32)
    if p.size < (length + 15) // 16:
        raise ValueError("gk_load_reference_2bit: packed holds fewer than ceil(length/16) words")
    if runs is None or len(runs) == 0:
        r, n_runs = None, 0
    else:
        r = np.ascontiguousarray(runs, dtype=np.uint64).reshape(-1, 2)
        n_runs = r.shape[0]
    st = lib().gk_load_reference_2bit(ctx, p.ctypes.data, length, layout,
                                      None if r is None else r.ctypes.data, n_runs)
    _check(ctx, st, "gk_load_reference_2bit")


def gk_reference_info(ctx) -> tuple[int, int]:
    n, u = ctypes.c_uint64(), ctypes.c_uint64()
    _check(ctx, lib().gk_reference_info(ctx, ctypes.byref(n), ctypes.byref(u)),
           "gk_reference_info")
    return int(n.value), int(u.value)


def gk_encode_reads(ctx, ascii, read_off, n_reads: int, pitch: int, rows: int, layout: int,
                    packed_out, len_out, has_n_out=None, stream=None) -> None:
    st = lib().gk_encode_reads(ctx, ptr(ascii), ptr(read_off), n_reads, pitch, rows, layout,
                               ptr(packed_out), ptr(len_out), ptr(has_n_out),
                               stream_handle(stream))
    _check(ctx, st, "gk_encode_reads")


def gk_set_option(ctx, option: int, value: int) -> None:
    _check(ctx, lib().gk_set_option(ctx, option, value), "gk_set_option")


def gk_get_option(ctx, option: int) -> int:
    v = ctypes.c_int64()
    _check(ctx, lib().gk_get_option(ctx, option, ctypes.byref(v)), "gk_get_option")
    return int(v.value)


def make_batch(*, n_reads, pitch, max_read_len, reads, read_len, pair_read, cand_pos, accept,
               est, n_pairs=None, e=None, e_uniform=0, read_has_n=None, accept_bits=None,
               read_layout=GK_READS_SPLIT, flags=0) -> gk_batch:
    b = gk_batch()
    b.flags = flags
    b.n_reads = n_reads
    b.pitch = pitch
    b.max_read_len = max_read_len
    b.e_uniform = e_uniform
    b.read_layout = read_layout
    b.reads = ptr(reads)
    b.read_len = ptr(read_len)
    b.read_has_n = ptr(read_has_n)
    b.n_pairs = n_pairs if n_pairs is not None else int(cand_pos.numel())
    b.pair_read = ptr(pair_read)
    b.cand_pos = ptr(cand_pos)
    b.e = ptr(e)
    b.accept = ptr(accept)
    b.est = ptr(est)
    b.accept_bits = ptr(accept_bits)
    return b


def gk_filter(ctx, batch: gk_batch, stream=None) -> None:
    _check(ctx, lib().gk_filter(ctx, ctypes.byref(batch), stream_handle(stream)), "gk_filter")


def gk_filter_ascii(ctx, batch: gk_batch, ascii, read_off, stream=None) -> None:
    """gk_filter with read i in ascii[read_off[i], read_off[i+1]) (device
    tensors), encoded in the same launch; pair i uses read i."""
    _check(ctx, lib().gk_filter_ascii(ctx, ctypes.byref(batch), ptr(ascii), ptr(read_off),
                                      stream_handle(stream)), "gk_filter_ascii")


def host_ptr(x):
    """Host address of a numpy array or a CPU torch tensor (pinned or not),
    or None."""
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        if x.is_cuda:
            raise ValueError("host buffer expected, got a device tensor")
        return x.data_ptr()
    return x.ctypes.data


def gk_filter_host(ctx, ascii, read_off, cand_pos, accept, est, *, max_read_len: int,
                   pair_read=None, e=None, e_uniform: int = 0, n_reads=None,
                   n_pairs=None, flags: int = 0, packed=None, read_len=None, read_has_n=None,
                   packed_layout: int = GK_READS_SPLIT) -> None:
    """Host buffers in, host results out (synchronous).  Arrays are
    contiguous numpy arrays of the ABI's dtypes, or CPU torch tensors (e.g.
    pinned byte buffers) with n_reads and n_pairs given.  With packed (host-
    encoded rows) and read_len, ascii and read_off are not used (may be None)."""
    if n_reads is None:
        n_reads = len(read_len) if packed is not None else len(read_off) - 1
    if n_pairs is None:
        n_pairs = len(cand_pos)
    b = gk_host_batch(n_reads=n_reads, max_read_len=max_read_len, ascii=host_ptr(ascii),
                      read_off=host_ptr(read_off), n_pairs=n_pairs,
                      pair_read=host_ptr(pair_read), cand_pos=host_ptr(cand_pos),
                      e=host_ptr(e), e_uniform=e_uniform, accept=host_ptr(accept),
                      est=host_ptr(est), flags=flags, packed=host_ptr(packed),
                      read_len=host_ptr(read_len), read_has_n=host_ptr(read_has_n),
                      packed_layout=packed_layout)
    _check(ctx, lib().gk_filter_host(ctx, ctypes.byref(b)), "gk_filter_host")


def gk_verify(ctx, batch: gk_batch, accept, dist, stream=None) -> None:
    """dist (device uint16, n_pairs) = min(edit distance, e + 1) for pairs
    whose device accept code is GK_ACCEPT (every pair when accept is None)."""
    _check(ctx, lib().gk_verify(ctx, ctypes.byref(batch), ptr(accept), ptr(dist),
                                stream_handle(stream)), "gk_verify")


def gk_filter_mixed(ctx, batch: gk_batch, stream=None) -> None:
    _check(ctx, lib().gk_filter_mixed(ctx, ctypes.byref(batch), stream_handle(stream)),
           "gk_filter_mixed")


def gk_filter_mixed_noalloc(ctx, batch: gk_batch, stream=None) -> None:
    _check(ctx, lib().gk_filter_mixed_noalloc(ctx, ctypes.byref(batch), stream_handle(stream)),
           "gk_filter_mixed_noalloc")


def gk_tune_mixed(ctx, batch: gk_batch, stream=None, sample_pairs: int = 0,
                  cache_path: str | None = None, report_cap: int = 1 << 16) -> str:
    """Returns the tuner's JSON report."""
    buf = ctypes.create_string_buffer(report_cap)
    st = lib().gk_tune_mixed(ctx, ctypes.byref(batch), stream_handle(stream), sample_pairs,
                             cache_path.encode() if cache_path else None, buf, report_cap)
    _check(ctx, st, "gk_tune_mixed")
    return buf.value.decode()


# ------------------------------------------------------------------ serving ---

def gk_server_start(ctx, device_budget_bytes: int, max_slots: int, max_read_len: int,
                    mode: int = GK_SERVER_BATCHED) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(ctx, lib().gk_server_start(ctx, device_budget_bytes, max_slots, max_read_len, mode,
                                      ctypes.byref(h)), "gk_server_start")
    return h


class Request:
    """A gk_request over host numpy arrays, which it keeps alive, with its own
    output arrays (accept uint8, est uint16)."""

    def __init__(self, reads, read_off, cand_pos, e: int, pair_read=None, t_arrival_us: int = 0,
                 accept=None, est=None):
        """accept / est: output arrays to fill (e.g. views of pinned memory);
        allocated here when None."""
        import numpy as np
        self.reads = np.ascontiguousarray(reads, dtype=np.uint8)
        self.read_off = np.ascontiguousarray(read_off, dtype=np.uint64)
        self.cand_pos = np.ascontiguousarray(cand_pos, dtype=np.uint32)
        self.pair_read = (np.ascontiguousarray(pair_read, dtype=np.uint32)
                          if pair_read is not None else None)
        n = len(self.cand_pos)
        self.accept = np.zeros(n, dtype=np.uint8) if accept is None else accept
        self.est = np.zeros(n, dtype=np.uint16) if est is None else est
        if (self.accept.dtype != np.uint8 or self.est.dtype != np.uint16 or
                len(self.accept) != n or len(self.est) != n or
                not self.accept.flags.c_contiguous or not self.est.flags.c_contiguous):
            raise ValueError("Request: accept must be uint8[n_pairs], est uint16[n_pairs]")
        r = gk_request()
        r.reads = self.reads.ctypes.data if self.reads.size else None
        r.read_off = self.read_off.ctypes.data
        r.n_reads = len(self.read_off) - 1
        r.e = e
        r.pair_read = self.pair_read.ctypes.data if self.pair_read is not None else None
        r.cand_pos = self.cand_pos.ctypes.data if n else None
        r.n_pairs = n
        r.accept = self.accept.ctypes.data if n else None
        r.est = self.est.ctypes.data if n else None
        r.t_arrival_us = t_arrival_us
        self.struct = r


def gk_server_submit(srv, req: Request) -> int:
    t = ctypes.c_uint64()
    st = lib().gk_server_submit(srv, ctypes.byref(req.struct), ctypes.byref(t))
    if st != GK_OK:
        raise GkError(st, "gk_server_submit")
    return int(t.value)


def gk_server_wait(srv, ticket: int, timeout_us: int = -1):
    """(status, gk_request_stats); status GK_ETIMEOUT leaves the ticket queued."""
    s = gk_request_stats()
    st = lib().gk_server_wait(srv, ticket, timeout_us, ctypes.byref(s))
    return int(st), s


def gk_server_counters(srv) -> tuple[int, int, int]:
    a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    st = lib().gk_server_counters(srv, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    if st != GK_OK:
        raise GkError(st, "gk_server_counters")
    return int(a.value), int(b.value), int(c.value)


def gk_server_tick_log(srv):
    """The server's completed ticks as a list of gk_tick_record."""
    n = ctypes.c_uint64()
    st = lib().gk_server_tick_log(srv, None, 0, ctypes.byref(n))
    if st != GK_OK:
        raise GkError(st, "gk_server_tick_log")
    buf = (gk_tick_record * max(1, n.value))()
    st = lib().gk_server_tick_log(srv, buf, n.value, ctypes.byref(n))
    if st != GK_OK:
        raise GkError(st, "gk_server_tick_log")
    return list(buf[:n.value])


def gk_server_stop(srv) -> None:
    st = lib().gk_server_stop(srv)
    if st != GK_OK:
        raise GkError(st, "gk_server_stop")


def gk_clock_us() -> int:
    return int(lib().gk_clock_us())

"""Helpers for GPU parity tests: run the same seeded pairs through the HIP
path (libgk) and through the oracle, element by element."""
from __future__ import annotations

import sys

import numpy as np

import oracle
from paper_2103_14978_amd import device, gk


def say(msg: str):
    """Name the case before each GPU step (flushed)."""
    print(msg, flush=True)
    sys.stdout.flush()


def run_gpu(ctx, ref_loaded_ascii, reads, read_off, pair_read, cand_pos, e, *, max_read_len=None,
            with_bits=False, load_ref=True, layout=gk.GK_READS_SPLIT, pairs_per_lane=None,
            identity_as_null=False):
    """Filter on the GPU.  e is an int (uniform) or a uint8 array per pair.
    identity_as_null: pass pair_read as NULL (requires pair_read[i] == i)."""
    if identity_as_null:
        assert np.array_equal(pair_read, np.arange(len(pair_read)))
        pair_read = None
    if load_ref:
        gk.gk_load_reference(ctx, ref_loaded_ascii)
    if pairs_per_lane is not None:
        gk.gk_set_option(ctx, gk.GK_OPT_PAIRS_PER_LANE, pairs_per_lane)
    dr = device.encode_reads(ctx, reads, read_off, max_len=max_read_len, layout=layout)
    per_pair = not np.isscalar(e) and not isinstance(e, int)
    dp = device.upload_pairs(pair_read, cand_pos, e if per_pair else None, with_bits=with_bits)
    b = device.batch_for(dr, dp, e_uniform=0 if per_pair else int(e), max_read_len=max_read_len)
    gk.gk_filter(ctx, b, None)
    import torch
    torch.cuda.synchronize()
    a, s = device.results(dp)
    bits = dp.accept_bits.cpu().numpy().view(np.uint64) if with_bits else None
    if pairs_per_lane is not None:
        gk.gk_set_option(ctx, gk.GK_OPT_PAIRS_PER_LANE, 0)
    return a, s, bits


def run_oracle(ref, reads, read_off, pair_read, cand_pos, e, threads=16):
    return oracle.filter_batch(reads, read_off, ref, pair_read, cand_pos, e, n_threads=threads)


def assert_same(a_gpu, s_gpu, a_ref, s_ref, label=""):
    bad = np.nonzero((a_gpu != a_ref) | (s_gpu != s_ref))[0]
    if len(bad):
        i = bad[0]
        raise AssertionError(f"{label}: {len(bad)} of {len(a_ref)} pairs differ; first at {i}: "
                             f"gpu=({a_gpu[i]},{s_gpu[i]}) oracle=({a_ref[i]},{s_ref[i]})")


def concat_reads(seqs):
    """list of bytes -> (uint8 ascii, uint64 offsets)"""
    lens = np.array([len(s) for s in seqs], dtype=np.uint64)
    off = np.zeros(len(seqs) + 1, dtype=np.uint64)
    np.cumsum(lens, out=off[1:])
    buf = np.frombuffer(b"".join(seqs), dtype=np.uint8) if seqs else np.zeros(0, np.uint8)
    return buf.copy(), off


def run_gpu_mixed(ctx, reads, read_off, pair_read, cand_pos, e, *, max_read_len, layout=0,
                  options=None, with_bits=False, repeats=1):
    """gk_filter_mixed on a resident reference.  options: {GK_OPT_*: value},
    reset to their defaults afterwards.  With repeats > 1 the call is
    replayed, the outputs cleared in between, and every replay returned."""
    import torch
    defaults = {gk.GK_OPT_MIXED_TILE: 4096, gk.GK_OPT_MIXED_PAIRS_PER_LANE: 1,
                gk.GK_OPT_MIXED_SORT_E: 1, gk.GK_OPT_MIXED_BLOCKS_PER_CU: 0,
                gk.GK_OPT_MIXED_GRAPH: 1}
    for k, v in (options or {}).items():
        gk.gk_set_option(ctx, k, v)
    try:
        dr = device.encode_reads(ctx, reads, read_off, max_len=max_read_len, layout=layout)
        per_pair = not np.isscalar(e) and not isinstance(e, int)
        dp = device.upload_pairs(pair_read, cand_pos, e if per_pair else None,
                                 with_bits=with_bits)
        b = device.batch_for(dr, dp, e_uniform=0 if per_pair else int(e),
                             max_read_len=max_read_len)
        out = []
        for _ in range(repeats):
            dp.accept.fill_(0xEE)
            dp.est.fill_(0x5A5A)
            if dp.accept_bits is not None:
                dp.accept_bits.fill_(-1)
            torch.cuda.synchronize()
            gk.gk_filter_mixed(ctx, b, None)
            torch.cuda.synchronize()
            a, s = device.results(dp)
            bits = dp.accept_bits.cpu().numpy().view(np.uint64) if with_bits else None
            out.append((a.copy(), s.copy(), bits))
        return out if repeats > 1 else out[0]
    finally:
        for k in (options or {}):
            gk.gk_set_option(ctx, k, defaults[k])


# ---- host-side 2-bit packing of a reference (for gk_load_reference_2bit) ----

_CODE = np.zeros(256, np.uint32)
BASE_MASK = np.zeros(256, bool)
for _ch, _c in zip(b"ACGT", range(4)):
    _CODE[_ch] = _CODE[_ch + 32] = _c
    BASE_MASK[_ch] = BASE_MASK[_ch + 32] = True


def pack_2bit(ascii, layout, rng, chunk=1 << 24):
    """16 bases per uint32 word in `layout` (GK_READS_SPLIT: low code bits in
    bits 0-15, high in 16-31; GK_READS_INTERLEAVED: base j at bits 2j, 2j+1).
    Unknown bases get random codes, which the loader must ignore."""
    a = np.asarray(ascii, np.uint8)
    out = np.zeros((len(a) + 15) // 16, np.uint32)
    j = np.arange(16, dtype=np.uint32)
    for first in range(0, len(a), chunk):
        part = a[first:first + chunk]
        codes = _CODE[part]
        unk = ~BASE_MASK[part]
        if unk.any():
            codes[unk] = rng.integers(0, 4, int(unk.sum()), dtype=np.uint32)
        n = (len(part) + 15) // 16 * 16
        c = np.zeros(n, np.uint32)
        c[:len(part)] = codes
        c = c.reshape(-1, 16)
        if layout == gk.GK_READS_SPLIT:
            w = ((c & 1) << j).sum(1) | ((c >> 1) << (16 + j)).sum(1)
        else:
            w = (c << (2 * j)).sum(1)
        out[first // 16:first // 16 + len(w)] = w
    return out


def unknown_runs(ascii):
    """Maximal runs of non-ACGT bytes as (start, length) pairs."""
    unk = ~BASE_MASK[np.asarray(ascii, np.uint8)]
    d = np.diff(np.concatenate([[0], unk.astype(np.int8), [0]]))
    starts = np.nonzero(d == 1)[0]
    ends = np.nonzero(d == -1)[0]
    return np.stack([starts, ends - starts], 1).astype(np.uint64)


def pack_reads_rows(reads, read_off, rows, layout):
    """Host encoding of reads for gk_filter_host's packed input: rows words
    per read, 16 bases per word in `layout`, code bits past each read's end
    zero; returns (packed uint32 [n_reads * rows], read_len uint16, has_n
    uint8).  Unknown bases get code 0 and set has_n."""
    reads = np.asarray(reads, np.uint8)
    off = np.asarray(read_off, np.int64)
    n = len(off) - 1
    lens = np.minimum(np.diff(off), 16 * rows)
    j = np.arange(16 * rows)
    valid = j[None, :] < lens[:, None]
    idx = np.where(valid, off[:-1, None] + j[None, :], 0)
    ch = np.where(valid, reads[idx], ord("A"))
    codes = np.where(valid, _CODE[ch], 0).astype(np.uint32).reshape(n, rows, 16)
    has_n = (valid & ~BASE_MASK[ch]).any(axis=1).astype(np.uint8)
    k = np.arange(16, dtype=np.uint32)
    if layout == gk.GK_READS_SPLIT:
        words = ((codes & 1) << k).sum(2) | ((codes >> 1) << (16 + k)).sum(2)
    else:
        words = (codes << (2 * k)).sum(2)
    return (np.ascontiguousarray(words.astype(np.uint32).reshape(-1)),
            np.diff(off).astype(np.uint16), has_n)

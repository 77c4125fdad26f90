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
            with_bits=False, load_ref=True):
    """Filter on the GPU.  e is an int (uniform) or a uint8 array per pair."""
    if load_ref:
        gk.gk_load_reference(ctx, ref_loaded_ascii)
    dr = device.encode_reads(ctx, reads, read_off, max_len=max_read_len)
    per_pair = not np.isscalar(e) and not isinstance(e, int)
    dp = device.upload_pairs(pair_read, cand_pos, e if per_pair else None, with_bits=with_bits)
    b = device.batch_for(dr, dp, e_uniform=0 if per_pair else int(e), max_read_len=max_read_len)
    gk.gk_filter(ctx, b, None)
    import torch
    torch.cuda.synchronize()
    a, s = device.results(dp)
    bits = dp.accept_bits.cpu().numpy().view(np.uint64) if with_bits else None
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

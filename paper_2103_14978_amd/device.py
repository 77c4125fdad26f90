"""Device-resident batches for libgk, built from host arrays with torch.

Plumbing only: torch allocates device memory and copies host arrays in; the
reads are 2-bit encoded by libgk's own kernel (gk_encode_reads) and filtered
by gk_filter.  Nothing of the filter is computed here.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import gk


def _dev(a: np.ndarray, device) -> torch.Tensor:
    a = np.ascontiguousarray(a)
    if not a.flags.writeable:
        a = a.copy()
    return torch.from_numpy(a).to(device, non_blocking=False)


def rows_for(max_len: int) -> int:
    """Rows of packed words (16 bases each) needed for reads up to max_len."""
    return max(1, (max_len + 15) // 16)


@dataclass
class DeviceReads:
    n_reads: int
    pitch: int
    max_len: int
    layout: int                 # gk.GK_READS_*
    packed: torch.Tensor        # uint32 [rows * pitch] (int32 storage)
    read_len: torch.Tensor      # uint16 (int16 storage)
    has_n: torch.Tensor         # uint8


def encode_reads(ctx, reads_ascii: np.ndarray, read_off: np.ndarray, *, max_len: int | None = None,
                 device="cuda", stream=None, pitch_align: int = 64,
                 layout: int = gk.GK_READS_SPLIT) -> DeviceReads:
    """Upload ASCII reads and encode them on the GPU (gk_encode_reads)."""
    read_off = np.ascontiguousarray(read_off, dtype=np.uint64)
    n = len(read_off) - 1
    if max_len is None:
        max_len = int(np.max(np.diff(read_off))) if n else 1
        max_len = max(1, min(max_len, gk.GK_MAX_READ_LEN))
    pitch = max(pitch_align, ((n + pitch_align - 1) // pitch_align) * pitch_align)
    rows = rows_for(max_len)
    ascii_d = _dev(np.ascontiguousarray(reads_ascii, dtype=np.uint8), device)
    if ascii_d.numel() == 0:
        ascii_d = torch.zeros(4, dtype=torch.uint8, device=device)
    off_d = _dev(read_off.view(np.int64), device)
    packed = torch.empty(rows * pitch, dtype=torch.int32, device=device)
    rl = torch.empty(max(n, 1), dtype=torch.int16, device=device)
    hn = torch.empty(max(n, 1), dtype=torch.uint8, device=device)
    gk.gk_encode_reads(ctx, ascii_d, off_d, n, pitch, rows, layout, packed, rl, hn, stream)
    torch.cuda.synchronize()
    del ascii_d, off_d
    return DeviceReads(n, pitch, max_len, layout, packed, rl, hn)


@dataclass
class DevicePairs:
    n_pairs: int
    pair_read: torch.Tensor | None  # uint32 (int32 storage); None = identity
    cand_pos: torch.Tensor      # uint32 (int32 storage)
    e: torch.Tensor | None      # uint8
    accept: torch.Tensor        # uint8
    est: torch.Tensor           # uint16 (int16 storage)
    accept_bits: torch.Tensor | None  # uint64 (int64 storage)


def upload_pairs(pair_read: np.ndarray | None, cand_pos: np.ndarray, e: np.ndarray | None = None,
                 *, device="cuda", with_bits: bool = False) -> DevicePairs:
    """pair_read None: pair i uses read i (one candidate per read)."""
    n = len(cand_pos)
    pr = (_dev(np.ascontiguousarray(pair_read, dtype=np.uint32).view(np.int32), device)
          if pair_read is not None else None)
    cp = _dev(np.ascontiguousarray(cand_pos, dtype=np.uint32).view(np.int32), device)
    ed = _dev(np.ascontiguousarray(e, dtype=np.uint8), device) if e is not None else None
    acc = torch.empty(max(n, 1), dtype=torch.uint8, device=device)
    est = torch.empty(max(n, 1), dtype=torch.int16, device=device)
    bits = torch.empty(max((n + 63) // 64, 1), dtype=torch.int64, device=device) if with_bits else None
    return DevicePairs(n, pr, cp, ed, acc, est, bits)


def batch_for(reads: DeviceReads, pairs: DevicePairs, *, e_uniform: int = 0,
              max_read_len: int | None = None, flags: int = 0) -> gk.gk_batch:
    return gk.make_batch(
        n_reads=reads.n_reads, pitch=reads.pitch,
        max_read_len=max_read_len if max_read_len is not None else reads.max_len,
        reads=reads.packed, read_len=reads.read_len, read_has_n=reads.has_n,
        n_pairs=pairs.n_pairs, pair_read=pairs.pair_read, cand_pos=pairs.cand_pos,
        e=pairs.e, e_uniform=e_uniform, accept=pairs.accept, est=pairs.est,
        accept_bits=pairs.accept_bits, read_layout=reads.layout, flags=flags)


def results(pairs: DevicePairs) -> tuple[np.ndarray, np.ndarray]:
    """(accept uint8, est uint16) copied back to the host."""
    n = pairs.n_pairs
    a = pairs.accept[:n].cpu().numpy()
    s = pairs.est[:n].cpu().numpy().view(np.uint16)
    return a, s

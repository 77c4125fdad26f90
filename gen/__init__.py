"""Seeded synthetic workloads for the GateKeeper filter (ctypes over gk_gen.c).

Shared by the tests (both the oracle side and the HIP side) and the benchmark.
Holds none of the filter's arithmetic: it produces ASCII sequences, integer
candidate positions, per-pair thresholds and a class label per pair.

The paper's own workloads (30M mrFAST/Minimap2/BWA-MEM candidate pairs from
real 100/150/250 bp reads, thresholds up to 10% of the read length; Sec. 4.1)
are not available; the configurations below stand in for them with the same
shapes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gk_gen.c")
LIB = os.path.join(HERE, "libgk_gen.so")

CLS_ORIGIN, CLS_BAND, CLS_SEEDED, CLS_RANDOM = 0, 1, 2, 3
CAND_ONE, CAND_GEOM, CAND_ZIPF = 0, 1, 2
EDIT_POISSON, EDIT_RATE = 0, 1
DECOY_RANDOM_POS, DECOY_SPLICE_KMER, DECOY_SEEDS = 0, 1, 2

GC_HUMANLIKE = 0.41


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared", "-pthread",
                               SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64),
        ("n_reads", ctypes.c_uint32),
        ("len_choices", ctypes.POINTER(ctypes.c_uint16)),
        ("n_len_choices", ctypes.c_uint32),
        ("cand_kind", ctypes.c_int),
        ("cand_param", ctypes.c_double),
        ("cand_cap", ctypes.c_uint32),
        ("true_frac", ctypes.c_double),
        ("edit_kind", ctypes.c_int),
        ("edit_param", ctypes.c_double),
        ("decoy_kind", ctypes.c_int),
        ("seed_k", ctypes.c_uint32),
        ("e_kind", ctypes.c_int),
        ("e_value", ctypes.c_uint32),
        ("e_frac", ctypes.c_double),
        ("gc", ctypes.c_double),
        ("band_cands", ctypes.c_int),
        ("n_true_first", ctypes.c_uint32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ctypes.CDLL(LIB)
        L.gkg_reference.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double,
                                    ctypes.c_uint64, ctypes.c_uint32]
        L.gkg_pairs_sizes.argtypes = [ctypes.POINTER(_Params), ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_uint32]
        L.gkg_pairs_fill.argtypes = [ctypes.POINTER(_Params), ctypes.c_void_p, ctypes.c_uint64,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_uint32]
        _lib = L
    return _lib


def default_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def reference(length: int, gc: float, seed: int, threads: int | None = None) -> np.ndarray:
    """i.i.d. reference of `length` ASCII bases (uint8) with GC fraction gc."""
    out = np.empty(length, dtype=np.uint8)
    lib().gkg_reference(out.ctypes.data, length, gc, seed, threads or default_threads())
    return out


@dataclass
class PairSet:
    """Reads (ASCII, concatenated) and their candidate pairs."""
    reads: np.ndarray          # uint8, concatenated ASCII
    read_off: np.ndarray       # uint64, n_reads + 1
    read_len: np.ndarray       # uint16, n_reads
    pair_read: np.ndarray      # uint32, n_pairs
    cand_pos: np.ndarray       # uint32, n_pairs
    e: np.ndarray              # uint8, n_pairs
    cls: np.ndarray            # uint8, n_pairs (CLS_*)
    meta: dict = field(default_factory=dict)

    @property
    def n_reads(self) -> int:
        return len(self.read_len)

    @property
    def n_pairs(self) -> int:
        return len(self.cand_pos)

    def read(self, i: int) -> bytes:
        return self.reads[self.read_off[i]:self.read_off[i + 1]].tobytes()

    def take_pairs(self, n: int) -> "PairSet":
        """The first n pairs (reads kept whole)."""
        return PairSet(self.reads, self.read_off, self.read_len, self.pair_read[:n],
                       self.cand_pos[:n], self.e[:n], self.cls[:n], dict(self.meta))


def pairs(ref: np.ndarray, *, seed: int, n_reads: int, lengths, cand_kind=CAND_ONE,
          cand_param=0.0, cand_cap=1, true_frac=0.5, edit_kind=EDIT_POISSON, edit_param=3.0,
          decoy_kind=DECOY_RANDOM_POS, seed_k=12, e_value=0, e_frac=None, gc=GC_HUMANLIKE,
          band_cands=False, n_true_first=0, threads: int | None = None) -> PairSet:
    lens = np.ascontiguousarray(np.asarray(lengths, dtype=np.uint16))
    p = _Params()
    p.seed = seed
    p.n_reads = n_reads
    p.len_choices = lens.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16))
    p.n_len_choices = len(lens)
    p.cand_kind = cand_kind
    p.cand_param = cand_param
    p.cand_cap = max(1, cand_cap)
    p.true_frac = true_frac
    p.edit_kind = edit_kind
    p.edit_param = edit_param
    p.decoy_kind = decoy_kind
    p.seed_k = seed_k
    p.e_kind = 0 if e_frac is None else 1
    p.e_value = e_value
    p.e_frac = 0.0 if e_frac is None else e_frac
    p.gc = gc
    p.band_cands = int(band_cands)
    p.n_true_first = n_true_first
    t = threads or default_threads()
    read_len = np.empty(n_reads, dtype=np.uint16)
    n_cand = np.empty(n_reads, dtype=np.uint32)
    lib().gkg_pairs_sizes(ctypes.byref(p), read_len.ctypes.data, n_cand.ctypes.data, t)
    read_off = np.zeros(n_reads + 1, dtype=np.uint64)
    np.cumsum(read_len, out=read_off[1:])
    pair_off = np.zeros(n_reads + 1, dtype=np.uint64)
    np.cumsum(n_cand, out=pair_off[1:])
    n_pairs = int(pair_off[-1])
    reads = np.empty(int(read_off[-1]), dtype=np.uint8)
    pair_read = np.empty(n_pairs, dtype=np.uint32)
    cand_pos = np.empty(n_pairs, dtype=np.uint32)
    pe = np.empty(n_pairs, dtype=np.uint8)
    cls = np.empty(n_pairs, dtype=np.uint8)
    ref = np.ascontiguousarray(ref, dtype=np.uint8)
    lib().gkg_pairs_fill(ctypes.byref(p), ref.ctypes.data, len(ref), read_off.ctypes.data,
                         pair_off.ctypes.data, reads.ctypes.data, pair_read.ctypes.data,
                         cand_pos.ctypes.data, pe.ctypes.data, cls.ctypes.data, t)
    return PairSet(reads, read_off, read_len, pair_read, cand_pos, pe, cls)


# ---------------------------------------------------------------- configs ---
#
# Config 0: plain filter, CPU-sized.
# Config 1: plain filter at paper-like scale (100 bp, e swept 0..10).
# Config 2: longer reads (150 / 250 bp), several candidates per read.
# Config 3: mixed batch (lengths 64..300, per-pair e, Zipf candidates).
# Config 4: served requests over a 3.1 Gbp reference.

REF_SEED = {0: 1000, 1: 1001, 2: 1001, 3: 1001, 4: 1004}
PAIR_SEED = {0: 2000, 1: 2001, 2: 2002, 3: 2003, 4: 3004}


def c0_reference() -> np.ndarray:
    """1 Mbp uniform i.i.d. ACGT reference."""
    return reference(1_000_000, 0.5, REF_SEED[0])


def c0_pairs(ref: np.ndarray, n_reads: int = 10_000) -> PairSet:
    """10,000 reads of 100 bp, each copied from a uniform origin with a
    Poisson(3) number of edits (70% substitution, 15% 1-3 bp insertion, 15%
    1-3 bp deletion).  The first half is paired with its origin, the second
    half with an independent uniform position.  e = 2."""
    ps = pairs(ref, seed=PAIR_SEED[0], n_reads=n_reads, lengths=[100],
               edit_kind=EDIT_POISSON, edit_param=3.0, decoy_kind=DECOY_RANDOM_POS,
               e_value=2, n_true_first=n_reads // 2, true_frac=0.5)
    ps.meta.update(config=0, e=2)
    return ps


def c1_reference(length: int = 100_000_000) -> np.ndarray:
    """100 Mbp i.i.d. reference with 41% GC."""
    return reference(length, GC_HUMANLIKE, REF_SEED[1])


def c1_pairs(ref: np.ndarray, e: int, n_pairs: int = 1 << 24) -> PairSet:
    """n_pairs 100 bp reads, one candidate each.  30% true origins with
    Poisson(e) edits; 70% decoys: an unrelated genome read with the exact
    12-mer ref[q+o, q+o+12) spliced in at offset o, paired with q."""
    ps = pairs(ref, seed=PAIR_SEED[1] + 100 * e, n_reads=n_pairs, lengths=[100],
               true_frac=0.3, edit_kind=EDIT_POISSON, edit_param=float(e),
               decoy_kind=DECOY_SPLICE_KMER, seed_k=12, e_value=e)
    ps.meta.update(config=1, e=e)
    return ps


def _solve_true_frac(mean_c: float, mean_extra: float, decoy_share: float = 0.6) -> float:
    """Fraction t of true reads giving the wanted share of decoy pairs, when a
    true read contributes mean_extra random (non-band) candidates on average."""
    t = (1.0 - decoy_share) * mean_c / max(mean_c - mean_extra, 1e-9)
    return float(min(max(t, 0.0), 1.0))


def _geom_pmf(p: float, cap: int) -> np.ndarray:
    c = np.arange(1, cap + 1, dtype=np.float64)
    pmf = p * (1 - p) ** (c - 1)
    pmf[-1] = (1 - p) ** (cap - 1)
    return pmf


def _zipf_pmf(s: float, cap: int) -> np.ndarray:
    c = np.arange(1, cap + 1, dtype=np.float64)
    w = c ** (-s)
    return w / w.sum()


def _true_frac_for(pmf: np.ndarray, e_values: np.ndarray) -> float:
    c = np.arange(1, len(pmf) + 1, dtype=np.float64)
    mean_c = float((pmf * c).sum())
    extras = [float((pmf * np.maximum(0.0, c - 1 - 2 * e)).sum()) for e in e_values]
    return _solve_true_frac(mean_c, float(np.mean(extras)))


def c2_pairs(ref: np.ndarray, m: int, e: int, n_pairs: int = 1 << 25) -> PairSet:
    """Reads of m bp (150 or 250) with 1..64 candidates (geometric, mean 8).
    True reads carry edits at a per-base rate uniform in [0, 1.2e/m]; their
    first candidate is the origin, then shifts of the origin by up to e
    bases, then random positions.  Decoy reads are random sequence carrying
    exact 16-mers copied from reference sites (candidate = site - offset).
    The true fraction is set so that 60% of pairs are decoys in expectation."""
    pmf = _geom_pmf(1 / 8, 64)
    t = _true_frac_for(pmf, np.array([e]))
    n_reads = int(n_pairs / float((pmf * np.arange(1, 65)).sum()) * 1.02) + 64
    ps = pairs(ref, seed=PAIR_SEED[2] + 7 * m + 100 * e, n_reads=n_reads, lengths=[m],
               cand_kind=CAND_GEOM, cand_param=1 / 8, cand_cap=64, true_frac=t,
               edit_kind=EDIT_RATE, edit_param=1.2, decoy_kind=DECOY_SEEDS, seed_k=16,
               e_value=e, band_cands=True)
    ps = ps.take_pairs(min(n_pairs, ps.n_pairs))
    ps.meta.update(config=2, m=m, e=e, true_frac=t)
    return ps


C3_LENGTHS = (64, 100, 150, 200, 250, 300)


def c3_pairs(ref: np.ndarray, n_pairs: int = 1 << 26) -> PairSet:
    """Mixed batch: read length uniform over {64,100,150,200,250,300}, e per
    pair uniform over 0..floor(0.1 m), Zipf(1.5) candidates per read capped at
    1024; pair mix as config 2."""
    pmf = _zipf_pmf(1.5, 1024)
    e_vals = np.concatenate([np.arange(0, int(0.1 * m) + 1) for m in C3_LENGTHS])
    t = _true_frac_for(pmf, e_vals)
    mean_c = float((pmf * np.arange(1, 1025)).sum())
    n_reads = int(n_pairs / mean_c * 1.05) + 1024
    ps = pairs(ref, seed=PAIR_SEED[3], n_reads=n_reads, lengths=list(C3_LENGTHS),
               cand_kind=CAND_ZIPF, cand_param=1.5, cand_cap=1024, true_frac=t,
               edit_kind=EDIT_RATE, edit_param=1.2, decoy_kind=DECOY_SEEDS, seed_k=16,
               e_frac=0.1, band_cands=True)
    ps = ps.take_pairs(min(n_pairs, ps.n_pairs))
    ps.meta.update(config=3, true_frac=t)
    return ps


def c4_reference(length: int = 3_100_000_000) -> np.ndarray:
    """3.1 Gbp i.i.d. reference with 41% GC."""
    return reference(length, GC_HUMANLIKE, REF_SEED[4])


def c4_request(ref: np.ndarray, index: int) -> PairSet:
    """One served request: n pairs log-uniform on [1e3, 1e6], one read length
    uniform on 100..250, one e uniform on 0..floor(0.1 m); reads with
    geometric(1/8) <= 64 candidates; pair mix as config 2."""
    rng = np.random.Generator(np.random.PCG64(PAIR_SEED[4] * 1_000_003 + index))
    n = int(np.exp(rng.uniform(np.log(1e3), np.log(1e6))))
    m = int(rng.integers(100, 251))
    e = int(rng.integers(0, int(0.1 * m) + 1))
    pmf = _geom_pmf(1 / 8, 64)
    t = _true_frac_for(pmf, np.array([e]))
    n_reads = int(n / 8.0 * 1.1) + 64
    ps = pairs(ref, seed=PAIR_SEED[4] + 1_000_000 * (index + 1), n_reads=n_reads, lengths=[m],
               cand_kind=CAND_GEOM, cand_param=1 / 8, cand_cap=64, true_frac=t,
               edit_kind=EDIT_RATE, edit_param=1.2, decoy_kind=DECOY_SEEDS, seed_k=16,
               e_value=e, band_cands=True)
    ps = ps.take_pairs(min(n, ps.n_pairs))
    ps.meta.update(config=4, m=m, e=e, request=index)
    return ps

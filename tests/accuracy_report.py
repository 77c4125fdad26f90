#!/usr/bin/env python3
"""False-accept / false-reject report of the filter against edit distance.

For each workload and threshold e, on a seeded sample of its pairs, the
oracle filters every pair (with the GPU version's leading/trailing
refinement of Sec. 3.4; without it, which is the GateKeeper-FPGA behaviour;
and with the Hamming fast path, a variant the paper does not describe) and the banded Levenshtein distance (unit-cost global alignment
of the read and its window, capped at e + 1) decides which pairs truly lie
within e edits.  As in Sec. 4.4 and Sec. 5.1:
    FA = accepted although lev > e,   FA rate = FA / #(lev > e)
    FR = rejected although lev <= e,  FR rate = FR / #(lev <= e)
Pairs with unknown bases or windows past the reference end are passed
undefined and counted apart.  The GPU path is bit-exact with the oracle, so
these figures hold for it too.  Calls only the oracle and the input
generators; prints a markdown table.

    python tests/accuracy_report.py [--sample 262144] [--threads 16]
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import gen      # noqa: E402
import oracle   # noqa: E402

NO_REFINE = 1
HAMMING = 2


def row(label, ref, ps, e, threads):
    e_arr = e if isinstance(e, np.ndarray) else None
    cap = int(e_arr.max()) if e_arr is not None else int(e)
    a, _ = oracle.filter_batch(ps.reads, ps.read_off, ref, ps.pair_read, ps.cand_pos, e,
                               n_threads=threads)
    a0, _ = oracle.filter_batch(ps.reads, ps.read_off, ref, ps.pair_read, ps.cand_pos, e,
                                flags=NO_REFINE, n_threads=threads)
    ah, _ = oracle.filter_batch(ps.reads, ps.read_off, ref, ps.pair_read, ps.cand_pos, e,
                                flags=HAMMING, n_threads=threads)
    lev = oracle.levenshtein_batch(ps.reads, ps.read_off, ref, ps.pair_read, ps.cand_pos, cap,
                                   n_threads=threads).astype(np.int64)
    ee = e_arr.astype(np.int64) if e_arr is not None else int(e)
    defined = a <= 1
    within = defined & (lev <= ee)
    beyond = defined & (lev > ee)
    fa = int(np.sum(beyond & (a == 1)))
    fr = int(np.sum(within & (a == 0)))
    fa0 = int(np.sum(beyond & (a0 == 1)))
    fr0 = int(np.sum(within & (a0 == 0)))
    fah = int(np.sum(beyond & (ah == 1)))
    frh = int(np.sum(within & (ah == 0)))
    nb, nw = int(beyond.sum()), int(within.sum())

    def rate(x, n):
        return f"{x / n:.4f}" if n else "-"
    return (f"| {label} | {ps.n_pairs} | {int((~defined).sum())} | {nw} | {nb} | "
            f"{fa} ({rate(fa, nb)}) | {fr} ({rate(fr, nw)}) | {fa0} ({rate(fa0, nb)}) | "
            f"{fr0} ({rate(fr0, nw)}) | {fah} ({rate(fah, nb)}) | {frh} ({rate(frh, nw)}) |")


class _Pooled:
    """Several pair sets as one: reads concatenated, pair_read re-based."""

    def __init__(self, reads, read_off, pair_read, cand_pos):
        self.reads, self.read_off = reads, read_off
        self.pair_read, self.cand_pos = pair_read, cand_pos
        self.n_pairs = len(cand_pos)


def concat_sets(parts):
    reads = np.concatenate([p.reads for p in parts])
    offs, prs, base_r, base_b = [np.zeros(1, np.uint64)], [], 0, 0
    for p in parts:
        offs.append(p.read_off[1:].astype(np.uint64) + np.uint64(base_b))
        prs.append(p.pair_read.astype(np.int64) + base_r)
        base_r += len(p.read_off) - 1
        base_b += int(p.read_off[-1])
    return _Pooled(reads, np.concatenate(offs), np.concatenate(prs).astype(np.uint32),
                   np.concatenate([p.cand_pos for p in parts]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sample", type=int, default=1 << 18)
    ap.add_argument("--threads", type=int, default=gen.default_threads())
    args = ap.parse_args()
    n, th = args.sample, args.threads
    t0 = time.time()
    print("| workload | pairs | undefined | lev <= e | lev > e | FA (rate) | FR (rate) | "
          "FA without refinement | FR without refinement | FA with Hamming fast path | "
          "FR with Hamming fast path |")
    print("|---|---|---|---|---|---|---|---|---|---|---|")
    ref0 = gen.c0_reference()
    ps = gen.c0_pairs(ref0)
    for e in (0, 1, 2, 3, 5):
        print(row(f"config 0 (100 bp), e={e}", ref0, ps, e, th), flush=True)
    ref = gen.c1_reference()
    for e in range(0, 11):
        print(row(f"config 1 (100 bp), e={e}", ref, gen.c1_pairs(ref, e, n_pairs=n), e, th),
              flush=True)
    for m, es in ((150, (3, 7, 15)), (250, (5, 12, 25))):
        for e in es:
            ps = gen.c2_pairs(ref, m, e, n_pairs=n // 2)
            print(row(f"config 2 ({m} bp), e={e}", ref, ps, e, th), flush=True)
    ps = gen.c3_pairs(ref, n_pairs=n)
    print(row("config 3 (64-300 bp), e per pair", ref, ps, ps.e, th), flush=True)
    del ref, ps
    # config 4: the served pool's first 16 requests (each its own length and
    # e) over the 3.1 Gbp reference, at most n/32 seeded pairs of each
    ref4 = gen.c4_reference()
    rng = np.random.default_rng(4004)
    parts = []
    for k in range(16):
        r = gen.c4_request(ref4, k)
        keep = np.sort(rng.choice(r.n_pairs, size=min(r.n_pairs, n // 32), replace=False))
        parts.append((_Pooled(r.reads, r.read_off, r.pair_read[keep], r.cand_pos[keep]),
                      r.meta["e"]))
    print(row("config 4 (100-250 bp, 16 requests), e per request", ref4,
              concat_sets([p for p, _ in parts]),
              np.concatenate([np.full(p.n_pairs, e, np.uint8) for p, e in parts]), th),
          flush=True)
    print(f"\n{time.time() - t0:.0f} s on {th} threads, sample {n} pairs per row "
          f"(config 2: {n // 2})", file=sys.stderr)


if __name__ == "__main__":
    main()

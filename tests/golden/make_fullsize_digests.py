"""Writes fullsize_digests.json: SHA-256 digests of the oracle's outputs
(accept codes, then estimates as little-endian uint16) on every pair of the
full-size workloads, so that the GPU tests can check every pair of a run at
those sizes without running the oracle on the GPU host.  Calls only the
seeded generators (gen) and the oracle.  Takes about half an hour on 8 cores.

    python tests/golden/make_fullsize_digests.py [--threads N]
"""
import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import gen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "fullsize_digests.json")

# (label, workload) for every full-size point the GPU tests filter
POINTS = ([("config2 m=150 e=%d" % e, ("c2", 150, e)) for e in (3, 7, 15)] +
          [("config2 m=250 e=%d" % e, ("c2", 250, e)) for e in (5, 12, 25)] +
          [("config3", ("c3",))])


def digest(a, s) -> str:
    h = hashlib.sha256()
    h.update(a.astype("u1").tobytes())
    h.update(s.astype("<u2").tobytes())
    return h.hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    ref = gen.c1_reference()
    out = {"what": "sha256 of the oracle's accept codes (u8) followed by its estimates "
                   "(little-endian u16), every pair, in pair order",
           "points": {}}
    for label, w in POINTS:
        t = time.time()
        if w[0] == "c2":
            ps = gen.c2_pairs(ref, w[1], w[2])
            e = w[2]
        else:
            ps = gen.c3_pairs(ref)
            e = ps.e
        a, s = oracle.filter_batch(ps.reads, ps.read_off, ref, ps.pair_read, ps.cand_pos, e,
                                   n_threads=args.threads)
        out["points"][label] = {"n_pairs": int(ps.n_pairs), "sha256": digest(a, s),
                                "accepted": int((a == 1).sum())}
        print(f"{label}: {ps.n_pairs} pairs, {time.time() - t:.0f} s", flush=True)
        with open(OUT, "w") as f:
            json.dump(out, f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main()

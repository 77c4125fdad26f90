"""GPU parity: libgk's HIP filter against the oracle, bit-exact on every pair.

Results are integers (accept code and edit estimate), so the bar is exact
equality element by element."""
import itertools

import numpy as np
import pytest

import gen
from gpu_cases import assert_same, concat_reads, run_gpu, run_oracle, say

pytestmark = pytest.mark.gpu


def test_config0_full(gkctx):
    """Config 0 in full: 1 Mbp uniform reference, 10,000 pairs of 100 bp, e=2."""
    say("case: config0 full (10,000 pairs, 100bp, e=2)")
    ref = gen.c0_reference()
    ps = gen.c0_pairs(ref)
    a, s, bits = run_gpu(gkctx, ref, ps.reads, ps.read_off, ps.pair_read, ps.cand_pos, 2,
                         with_bits=True)
    ra, rs = run_oracle(ref, ps.reads, ps.read_off, ps.pair_read, ps.cand_pos, 2)
    assert_same(a, s, ra, rs, "config0")
    # accept bits: 1 for ACCEPT or UNDEFINED
    want = (ra == 1) | (ra == 2)
    got = np.unpackbits(bits.view(np.uint8), bitorder="little")[:len(ra)].astype(bool)
    assert np.array_equal(got, want)


def _all_words(m):
    return [bytes(t) for t in itertools.product(b"ACGT", repeat=m)]


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_exhaustive_small(gkctx, m):
    """Every (read, window) pair of length m over ACGT, e = 0..m+1."""
    words = _all_words(m)
    n = len(words)
    ref = np.frombuffer(b"".join(words), dtype=np.uint8).copy()
    reads, off = concat_reads(words)
    ri, wi = np.meshgrid(np.arange(n, dtype=np.uint32), np.arange(n, dtype=np.uint32),
                         indexing="ij")
    pr, pos = ri.reshape(-1), (wi.reshape(-1) * m).astype(np.uint32)
    loaded = False
    for e in range(0, m + 2):
        say(f"case: exhaustive m={m} e={e} pairs={len(pr)}")
        a, s, _ = run_gpu(gkctx, ref, reads, off, pr, pos, e, load_ref=not loaded)
        loaded = True
        ra, rs = run_oracle(ref, reads, off, pr, pos, e)
        assert_same(a, s, ra, rs, f"exhaustive m={m} e={e}")


def test_exhaustive_m6(gkctx):
    """All 4^6 x 4^6 pairs (16.7M) at e = 1 and 3."""
    m = 6
    words = _all_words(m)
    n = len(words)
    ref = np.frombuffer(b"".join(words), dtype=np.uint8).copy()
    reads, off = concat_reads(words)
    pr = np.repeat(np.arange(n, dtype=np.uint32), n)
    pos = np.tile(np.arange(n, dtype=np.uint32) * m, n)
    loaded = False
    for e in (1, 3):
        say(f"case: exhaustive m=6 e={e}")
        a, s, _ = run_gpu(gkctx, ref, reads, off, pr, pos, e, load_ref=not loaded)
        loaded = True
        ra, rs = run_oracle(ref, reads, off, pr, pos, e)
        assert_same(a, s, ra, rs, f"exhaustive m=6 e={e}")


LENGTHS = list(range(1, 41)) + [63, 64, 65, 95, 96, 97, 100, 127, 128, 129, 150, 159, 160, 161,
                                 191, 192, 193, 250, 255, 256, 257, 300, 480, 500, 511, 512]


def _sweep_pairs(ref, m, n_reads, rng):
    """Reads near their window (a few edits) and random reads, at positions
    covering every residue mod 32."""
    L = len(ref)
    seqs, pr, pos = [], [], []
    for i in range(n_reads):
        p = int(rng.integers(0, L - m - 8))
        p = (p & ~31) + (i % 32)
        if p + m > L:
            p = L - m
        s = bytearray(ref[p:p + m].tobytes())
        kind = i % 4
        if kind == 1:
            for _ in range(int(rng.integers(1, 4))):
                s[int(rng.integers(0, m))] = b"ACGT"[int(rng.integers(0, 4))]
        elif kind == 2:
            d = int(rng.integers(1, 4))
            s = bytearray(ref[p + d:p + d + m].tobytes())
        elif kind == 3:
            s = bytearray(rng.choice(np.frombuffer(b"ACGT", np.uint8), m).tobytes())
        seqs.append(bytes(s))
        pr.append(i)
        pos.append(p)
    reads, off = concat_reads(seqs)
    return reads, off, np.array(pr, np.uint32), np.array(pos, np.uint32)


def _e_values(m):
    return sorted({0, 1, 2, 5, m // 10, 31, 32, 40, max(m - 1, 0), m, min(m + 3, 255)})


def test_length_sweep_uniform_launch(gkctx):
    """Word-boundary lengths, each in its own launch sized for it."""
    rng = np.random.default_rng(77)
    ref = gen.reference(200_000, 0.45, 4242)
    from paper_2103_14978_amd import gk
    gk.gk_load_reference(gkctx, ref)
    for m in LENGTHS:
        reads, off, pr, pos = _sweep_pairs(ref, m, 256, rng)
        for e in _e_values(m):
            if e > 255:
                continue
            say(f"case: sweep m={m} e={e}")
            a, s, _ = run_gpu(gkctx, ref, reads, off, pr, pos, e, max_read_len=m, load_ref=False)
            ra, rs = run_oracle(ref, reads, off, pr, pos, e)
            assert_same(a, s, ra, rs, f"sweep m={m} e={e}")


def test_mixed_lengths_one_launch(gkctx):
    """Reads of many lengths and per-pair e in one launch for 512-base reads:
    shorter reads take the general path inside the same kernel."""
    rng = np.random.default_rng(78)
    ref = gen.reference(300_000, 0.41, 4243)
    seqs, prs, poss, es = [], [], [], []
    base = 0
    for m in LENGTHS:
        reads, off, pr, pos = _sweep_pairs(ref, m, 64, rng)
        for i in range(len(pr)):
            seqs.append(reads[off[i]:off[i + 1]].tobytes())
        prs.append(pr + base)
        poss.append(pos)
        es.append(rng.integers(0, min(m + 2, 60), len(pr)).astype(np.uint8))
        base += len(pr)
    reads, off = concat_reads(seqs)
    pr, pos, e = np.concatenate(prs), np.concatenate(poss), np.concatenate(es)
    say(f"case: mixed lengths one launch, {len(pr)} pairs")
    a, s, _ = run_gpu(gkctx, ref, reads, off, pr, pos, e, max_read_len=512)
    ra, rs = run_oracle(ref, reads, off, pr, pos, e)
    assert_same(a, s, ra, rs, "mixed lengths")


def test_config1_e_sweep_scaled(gkctx):
    """Config 1 generator at 2^16 pairs for every e in 0..10, all pairs."""
    ref = gen.c1_reference(20_000_000)
    from paper_2103_14978_amd import gk
    gk.gk_load_reference(gkctx, ref)
    for e in range(0, 11):
        ps = gen.c1_pairs(ref, e, n_pairs=1 << 16)
        say(f"case: config1 scaled e={e}")
        a, s, _ = run_gpu(gkctx, ref, ps.reads, ps.read_off, ps.pair_read, ps.cand_pos, e,
                          load_ref=False)
        ra, rs = run_oracle(ref, ps.reads, ps.read_off, ps.pair_read, ps.cand_pos, e)
        assert_same(a, s, ra, rs, f"config1 e={e}")


def test_config2_scaled(gkctx):
    """Config 2 generator (150 / 250 bp, several candidates per read) at 2^15
    pairs per (m, e)."""
    ref = gen.c1_reference(20_000_000)
    from paper_2103_14978_amd import gk
    gk.gk_load_reference(gkctx, ref)
    for m, es in ((150, (3, 7, 15)), (250, (5, 12, 25))):
        for e in es:
            ps = gen.c2_pairs(ref, m, e, n_pairs=1 << 15)
            say(f"case: config2 scaled m={m} e={e}")
            a, s, _ = run_gpu(gkctx, ref, ps.reads, ps.read_off, ps.pair_read, ps.cand_pos, e,
                              load_ref=False)
            ra, rs = run_oracle(ref, ps.reads, ps.read_off, ps.pair_read, ps.cand_pos, e)
            assert_same(a, s, ra, rs, f"config2 m={m} e={e}")


def test_config3_scaled_plain(gkctx):
    """Config 3 generator (mixed lengths, per-pair e) at 2^16 pairs through
    the plain filter in one launch."""
    ref = gen.c1_reference(20_000_000)
    ps = gen.c3_pairs(ref, n_pairs=1 << 16)
    say("case: config3 scaled, plain launch")
    a, s, _ = run_gpu(gkctx, ref, ps.reads, ps.read_off, ps.pair_read, ps.cand_pos, ps.e,
                      max_read_len=300)
    ra, rs = run_oracle(ref, ps.reads, ps.read_off, ps.pair_read, ps.cand_pos, ps.e)
    assert_same(a, s, ra, rs, "config3 plain")


@pytest.mark.parametrize("layout", [0, 1], ids=["split", "interleaved"])
@pytest.mark.parametrize("ppl", [0, 1, 2, 7, 65536])
def test_layouts_and_grid_shapes(gkctx, layout, ppl):
    """Both read layouts, and grids from one pair per lane to many pairs per
    lane with loads in flight, give the same bit-exact results: config 0
    pairs plus a mixed-length, per-pair-e set in one launch."""
    rng = np.random.default_rng(79)
    ref = gen.c0_reference()
    ps = gen.c0_pairs(ref, n_reads=3001)
    say(f"case: layout={layout} pairs_per_lane={ppl} config0")
    a, s, bits = run_gpu(gkctx, ref, ps.reads, ps.read_off, ps.pair_read, ps.cand_pos, 2,
                         layout=layout, pairs_per_lane=ppl, with_bits=True,
                         identity_as_null=(ppl % 2 == 1))
    ra, rs = run_oracle(ref, ps.reads, ps.read_off, ps.pair_read, ps.cand_pos, 2)
    assert_same(a, s, ra, rs, f"config0 layout={layout} ppl={ppl}")
    want = (ra == 1) | (ra == 2)
    got = np.unpackbits(bits.view(np.uint8), bitorder="little")[:len(ra)].astype(bool)
    assert np.array_equal(got, want)
    seqs, prs, poss, es = [], [], [], []
    for m in (5, 31, 33, 64, 100, 129, 200):
        reads, off, pr, pos = _sweep_pairs(ref, m, 97, rng)
        base = len(seqs)
        for i in range(len(pr)):
            seqs.append(reads[off[i]:off[i + 1]].tobytes())
        prs.append(pr + base)
        poss.append(pos)
        es.append(rng.integers(0, 40, len(pr)).astype(np.uint8))
    reads, off = concat_reads(seqs)
    pr, pos, e = np.concatenate(prs), np.concatenate(poss), np.concatenate(es)
    say(f"case: layout={layout} pairs_per_lane={ppl} mixed")
    a, s, _ = run_gpu(gkctx, ref, reads, off, pr, pos, e, max_read_len=200, layout=layout,
                      pairs_per_lane=ppl, load_ref=False)
    ra, rs = run_oracle(ref, reads, off, pr, pos, e)
    assert_same(a, s, ra, rs, f"mixed layout={layout} ppl={ppl}")

"""gk_load_reference_2bit: a reference handed over as 2-bit words plus
unknown-base runs gives the same resident state, and so the same results on
every pair, as the ASCII text it was packed from; both match the oracle."""
import ctypes

import numpy as np
import pytest

from gpu_cases import (BASE_MASK as _BASE, assert_same, concat_reads, pack_2bit, run_gpu,
                       run_oracle, say, unknown_runs)

pytestmark = pytest.mark.gpu

def make_reference(rng, L):
    ref = rng.choice(np.frombuffer(b"ACGTacgt", np.uint8), L).copy()
    # unknown runs: at the start, across word boundaries, single bases, at the end
    for s, l in ((0, 3), (31, 2), (63, 70), (500, 1), (502, 1), (4096, 33), (L - 5, 5)):
        if s + l <= L:
            ref[s:s + l] = np.frombuffer(b"N" * l, np.uint8)
    for s in rng.integers(0, L - 40, 20):
        ref[s:s + int(rng.integers(1, 40))] = ord("n")
    ref[777] = ord("R")
    return ref


def pairs_for(rng, ref, n):
    """Reads taken from the reference (some with substitutions) at random and
    at run-adjacent positions, lengths 1..300, windows up to the very end."""
    L = len(ref)
    seqs, pos = [], []
    runs = unknown_runs(ref)
    hot = np.concatenate([runs[:, 0], runs[:, 0] + runs[:, 1]]).astype(np.int64)
    for i in range(n):
        m = int(rng.integers(1, 301))
        if i % 3 == 0:
            p = int(hot[rng.integers(len(hot))]) + int(rng.integers(-m, 2))
        elif i % 7 == 0:
            p = L - m
        else:
            p = int(rng.integers(0, L - m + 1))
        p = min(max(p, 0), L - m)
        s = ref[p:p + m].copy()
        s[s == ord("N")] = ord("A")
        s[s == ord("n")] = ord("c")
        for q in rng.integers(0, m, int(rng.integers(0, 4))):
            s[q] = rng.choice(np.frombuffer(b"ACGT", np.uint8))
        seqs.append(s.tobytes())
        pos.append(rng.integers(0, L - m + 1) if i % 11 == 0 else p)
    reads, off = concat_reads(seqs)
    return reads, off, np.arange(n, dtype=np.uint32), np.array(pos, np.uint32)


@pytest.mark.parametrize("layout", [0, 1])
def test_2bit_equals_ascii_and_oracle(gkctx, layout):
    from paper_2103_14978_amd import gk
    rng = np.random.default_rng(40 + layout)
    L = 200_003
    ref = make_reference(rng, L)
    runs = unknown_runs(ref)
    n_unknown = int((~_BASE[ref]).sum())
    reads, off, pr, pos = pairs_for(rng, ref, 6000)
    e = rng.integers(0, 31, len(pr)).astype(np.uint8)
    say(f"case: 2bit layout={layout} L={L} runs={len(runs)}")
    ra, rs = run_oracle(ref, reads, off, pr, pos, e)
    assert np.any(ra == 2) and np.any(ra == 1) and np.any(ra == 0)

    gk.gk_load_reference(gkctx, ref)
    assert gk.gk_reference_info(gkctx) == (L, n_unknown)
    a1, s1, _ = run_gpu(gkctx, ref, reads, off, pr, pos, e, max_read_len=300, load_ref=False)
    assert_same(a1, s1, ra, rs, "ascii load")

    # The same runs, split in two, shuffled and overlapping, plus empty runs.
    half = runs.copy()
    half[:, 1] = (runs[:, 1] + 1) // 2
    tail = runs.copy()
    tail[:, 0] = runs[:, 0] + runs[:, 1] // 2
    tail[:, 1] = runs[:, 1] - runs[:, 1] // 2
    extra = np.array([[0, 0], [L - 1, 0]], np.uint64)
    all_runs = np.concatenate([half, tail, runs[::3], extra])
    all_runs = all_runs[rng.permutation(len(all_runs))]
    gk.gk_load_reference_2bit(gkctx, pack_2bit(ref, layout, rng), L, layout, all_runs)
    assert gk.gk_reference_info(gkctx) == (L, n_unknown)
    a2, s2, _ = run_gpu(gkctx, ref, reads, off, pr, pos, e, max_read_len=300, load_ref=False)
    assert_same(a2, s2, ra, rs, f"2bit load layout={layout}")


def test_2bit_small_lengths(gkctx):
    from paper_2103_14978_amd import gk
    rng = np.random.default_rng(47)
    for L in (1, 15, 16, 17, 31, 32, 33, 47, 64, 65, 1000):
        ref = rng.choice(np.frombuffer(b"ACGT", np.uint8), L).copy()
        if L > 10:
            ref[L // 2] = ord("N")
        say(f"case: 2bit small L={L}")
        gk.gk_load_reference_2bit(gkctx, pack_2bit(ref, 0, rng), L, 0, unknown_runs(ref))
        assert gk.gk_reference_info(gkctx) == (L, int((~_BASE[ref]).sum()))
        seqs = [ref[max(0, L - m):L].tobytes() for m in (1, 2, 5, 17, 40) if m <= L]
        seqs = [s.replace(b"N", b"A") for s in seqs] + [ref[:min(L, 33)].tobytes()]
        reads, off = concat_reads(seqs)
        pr = np.arange(len(seqs), dtype=np.uint32)
        pos = np.array([max(0, L - m) for m in (1, 2, 5, 17, 40) if m <= L] + [0], np.uint32)
        for e in (0, 2):
            a, s, _ = run_gpu(gkctx, ref, reads, off, pr, pos, e, max_read_len=64, load_ref=False)
            ra, rs = run_oracle(ref, reads, off, pr, pos, e)
            assert_same(a, s, ra, rs, f"2bit small L={L} e={e}")


def test_2bit_errors_keep_previous_reference(gkctx):
    from paper_2103_14978_amd import gk
    rng = np.random.default_rng(48)
    ref = rng.choice(np.frombuffer(b"ACGT", np.uint8), 5000).copy()
    gk.gk_load_reference(gkctx, ref)
    packed = pack_2bit(ref, 0, rng)
    L = gk.lib()
    cases = [
        (packed.ctypes.data, 5000, 7, None, 0, gk.GK_EINVAL),          # layout
        (None, 5000, 0, None, 0, gk.GK_EINVAL),                        # NULL words
        (packed.ctypes.data, 0, 0, None, 0, gk.GK_EINVAL),             # empty
        (packed.ctypes.data, 1 << 33, 0, None, 0, gk.GK_ERANGE),       # too long
        (packed.ctypes.data, 5000, 0, None, 1, gk.GK_EINVAL),          # NULL runs
    ]
    for words, n, layout, runs, nruns, want in cases:
        assert L.gk_load_reference_2bit(gkctx, words, n, layout, runs, nruns) == want
        assert gk.gk_reference_info(gkctx) == (5000, 0)
    for bad in ([[4999, 2]], [[5000, 1]], [[2**64 - 1, 2]]):
        r = np.array(bad, np.uint64)
        st = L.gk_load_reference_2bit(gkctx, packed.ctypes.data, 5000, 0, r.ctypes.data, 1)
        assert st == gk.GK_EINVAL, bad
        assert "past the reference end" in gk.gk_last_error(gkctx)
        assert gk.gk_reference_info(gkctx) == (5000, 0)
    # A run of length 0 anywhere is allowed, and the reference stays usable.
    r = np.array([[5000, 0]], np.uint64)
    assert L.gk_load_reference_2bit(gkctx, packed.ctypes.data, 5000, 0, r.ctypes.data, 1) == 0
    reads, off = concat_reads([ref[100:200].tobytes()])
    a, s, _ = run_gpu(gkctx, ref, reads, off, np.array([0], np.uint32),
                      np.array([100], np.uint32), 0, max_read_len=100, load_ref=False)
    assert (a[0], s[0]) == (1, 0)

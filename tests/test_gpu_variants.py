"""Variant semantics (gk_batch.flags): GK_FLAG_NO_REFINE gives the original
GateKeeper's results, GK_FLAG_HAMMING_FASTPATH the Hamming short-cut; both
through the plain, the mixed and the host-to-host entry points, against the
oracle run with the same flags."""
import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_cases import assert_same, say
from paper_2103_14978_amd import device, gk

pytestmark = pytest.mark.gpu

FLAGS = [gk.GK_FLAG_NO_REFINE, gk.GK_FLAG_HAMMING_FASTPATH,
         gk.GK_FLAG_NO_REFINE | gk.GK_FLAG_HAMMING_FASTPATH]


@pytest.fixture(scope="module")
def mixed_case():
    ref = gen.c1_reference(4_000_000)
    ps = gen.c3_pairs(ref, n_pairs=1 << 17)
    return ref, ps


@pytest.mark.parametrize("flags", FLAGS)
def test_variants_plain_and_mixed(gkctx, mixed_case, flags):
    ref, ps = mixed_case
    gk.gk_load_reference(gkctx, ref)
    say(f"case: variants flags={flags} pairs={ps.n_pairs}")
    ra, rs = oracle.filter_batch(ps.reads, ps.read_off, ref, ps.pair_read, ps.cand_pos, ps.e,
                                 flags=flags, n_threads=gen.default_threads())
    r0, _ = oracle.filter_batch(ps.reads, ps.read_off, ref, ps.pair_read, ps.cand_pos, ps.e,
                                n_threads=gen.default_threads())
    assert not np.array_equal(ra, r0)          # the variant changes some decisions
    layout = gk.GK_READS_INTERLEAVED if flags == FLAGS[-1] else gk.GK_READS_SPLIT
    dr = device.encode_reads(gkctx, ps.reads, ps.read_off, max_len=300, layout=layout)
    for mixed in (False, True):
        dp = device.upload_pairs(ps.pair_read, ps.cand_pos, ps.e)
        b = device.batch_for(dr, dp, max_read_len=300, flags=flags)
        (gk.gk_filter_mixed if mixed else gk.gk_filter)(gkctx, b, None)
        torch.cuda.synchronize()
        a, s = device.results(dp)
        assert_same(a, s, ra, rs, f"flags={flags} mixed={mixed}")
    # the default launch right after still gives the paper's results
    dp = device.upload_pairs(ps.pair_read, ps.cand_pos, ps.e)
    gk.gk_filter_mixed(gkctx, device.batch_for(dr, dp, max_read_len=300), None)
    torch.cuda.synchronize()
    a, _ = device.results(dp)
    assert np.array_equal(a, r0)


@pytest.mark.parametrize("flags", FLAGS)
def test_variants_host(gkctx, flags):
    ref = gen.c0_reference()
    gk.gk_load_reference(gkctx, ref)
    ps = gen.c0_pairs(ref)
    say(f"case: host variants flags={flags}")
    acc = np.zeros(ps.n_pairs, np.uint8)
    est = np.zeros(ps.n_pairs, np.uint16)
    gk.gk_filter_host(gkctx, ps.reads, ps.read_off, ps.cand_pos, acc, est, max_read_len=100,
                      e_uniform=5, flags=flags)
    ra, rs = oracle.filter_batch(ps.reads, ps.read_off, ref, ps.pair_read, ps.cand_pos, 5,
                                 flags=flags, n_threads=gen.default_threads())
    assert_same(acc, est, ra, rs, f"host flags={flags}")


def test_unknown_flags_rejected(gkctx):
    ref = gen.c0_reference()
    gk.gk_load_reference(gkctx, ref)
    ps = gen.c0_pairs(ref, n_reads=64)
    dr = device.encode_reads(gkctx, ps.reads, ps.read_off, max_len=100)
    dp = device.upload_pairs(None, ps.cand_pos)
    with pytest.raises(gk.GkError) as ei:
        gk.gk_filter(gkctx, device.batch_for(dr, dp, e_uniform=2, flags=4), None)
    assert ei.value.status == gk.GK_EINVAL



def _large_e_case(seed):
    """Pairs with e in 30..90 that the filter does not accept wholesale.

    At such thresholds almost every window passes, so the windows are cut from
    a planted stretch of A/C bases and each read carries a block of G/T bases
    of length e..3e+8 (at the start, the end or inside).  Block bases mismatch
    the window under every shift; the AND keeps about (block - 2e) of them, more
    at a read end, where the vacated positions (compared with 'A') decide
    whether refinement matters.  This splits decisions near e."""
    from gpu_cases import concat_reads
    rng = np.random.default_rng(seed)
    ref = gen.reference(400_000, 0.41, 4244)
    lo, hi = 200_000, 212_000
    ref[lo:hi] = np.frombuffer(b"AC", np.uint8)[rng.integers(0, 2, hi - lo)]
    seqs, pos, es = [], [], []
    for m in (100, 128, 161, 256, 300):
        for i in range(300):
            e = int(rng.integers(30, min(90, (m - 4) // 3) + 1))
            p = int(rng.integers(lo, hi - m))
            s = ref[p:p + m].copy()
            k = int(rng.integers(e, min(m, 3 * e + 8) + 1))
            at = (0, m - k, int(rng.integers(0, m - k + 1)))[i % 3]
            s[at:at + k] = np.frombuffer(b"GT", np.uint8)[rng.integers(0, 2, k)]
            seqs.append(s.tobytes())
            pos.append(p + int(rng.integers(-2, 3)) * (i % 4 == 0))
            es.append(e)
    reads, off = concat_reads(seqs)
    return (ref, reads, off, np.arange(len(seqs), dtype=np.uint32),
            np.array(pos, np.uint32), np.array(es, np.uint8))


@pytest.mark.parametrize("flags", [0] + FLAGS)
def test_variants_large_e_general_path(gkctx, flags):
    """Thresholds of 30..90 (whole-word shifts of the general path, and the
    mixed launch's residual pass), by default and under each variant."""
    ref, reads, off, pr, pos, e = _large_e_case(300 + flags)
    gk.gk_load_reference(gkctx, ref)
    say(f"case: variants large e flags={flags} pairs={len(pr)}")
    ra, rs = oracle.filter_batch(reads, off, ref, pr, pos, e, flags=flags,
                                 n_threads=gen.default_threads())
    r0, _ = oracle.filter_batch(reads, off, ref, pr, pos, e,
                                n_threads=gen.default_threads())
    assert 0.2 < np.mean(ra == gk.GK_ACCEPT) < 0.8
    if flags & gk.GK_FLAG_NO_REFINE:
        assert not np.array_equal(ra, r0)
    dr = device.encode_reads(gkctx, reads, off, max_len=300)
    for mixed in (False, True):
        dp = device.upload_pairs(pr, pos, e)
        b = device.batch_for(dr, dp, max_read_len=300, flags=flags)
        (gk.gk_filter_mixed if mixed else gk.gk_filter)(gkctx, b, None)
        torch.cuda.synchronize()
        a, s = device.results(dp)
        assert_same(a, s, ra, rs, f"large e flags={flags} mixed={mixed}")

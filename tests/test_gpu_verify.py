"""gk_verify: the edit distance of the verification step the filter precedes,
capped at e + 1, against the oracle's banded dynamic programme."""
import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_cases import concat_reads, say
from paper_2103_14978_amd import device, gk

pytestmark = pytest.mark.gpu


def oracle_dist(ref, reads, off, pair_read, cand_pos, e):
    """min(lev, e + 1) per pair, grouped by threshold."""
    e = np.asarray(e)
    out = np.zeros(len(cand_pos), np.uint16)
    for v in np.unique(e):
        idx = np.nonzero(e == v)[0]
        out[idx] = oracle.levenshtein_batch(reads, off, ref, pair_read[idx], cand_pos[idx],
                                            int(v), n_threads=gen.default_threads())
    return out


def edited_pairs(rng, ref, n, max_len=300, max_e=31, min_len=1):
    """Reads copied from the reference with random substitutions and 1-3 base
    insertions / deletions, paired with their origin or a nearby shift."""
    seqs, pos = [], []
    L = len(ref)
    for _ in range(n):
        m = int(rng.integers(min_len, max_len + 1))
        p = int(rng.integers(0, L - m - 8))
        src = list(ref[p:p + m + 8].tobytes())
        for _ in range(int(rng.poisson(1 + m / 25))):
            q = int(rng.integers(0, len(src)))
            k = rng.random()
            if k < 0.6:
                src[q] = int(rng.choice(np.frombuffer(b"ACGT", np.uint8)))
            elif k < 0.8:
                for _ in range(int(rng.integers(1, 4))):
                    src.insert(q, int(rng.choice(np.frombuffer(b"ACGT", np.uint8))))
            elif len(src) > m + 3:
                del src[q:q + int(rng.integers(1, 4))]
        seqs.append(bytes(src[:m]))
        pos.append(min(max(p + int(rng.integers(-2, 3)), 0), L - m))
    reads, off = concat_reads(seqs)
    e = rng.integers(0, max_e + 1, n).astype(np.uint8)
    return reads, off, np.arange(n, dtype=np.uint32), np.array(pos, np.uint32), e


def verify(ctx, reads, off, pr, pos, e, max_len, accept=None, layout=0, e_uniform=None):
    """e: per-pair thresholds, or None with e_uniform for the whole batch."""
    dr = device.encode_reads(ctx, reads, off, max_len=max_len, layout=layout)
    dp = device.upload_pairs(pr, pos, e)
    b = device.batch_for(dr, dp, max_read_len=max_len,
                         e_uniform=e_uniform if e_uniform is not None else 0)
    dist = torch.empty(len(pos), dtype=torch.int16, device="cuda")
    acc = None if accept is None else torch.from_numpy(accept).cuda()
    gk.gk_verify(ctx, b, acc, dist, None)
    torch.cuda.synchronize()
    return dist.cpu().numpy().view(np.uint16)


@pytest.mark.parametrize("max_len", [64, 150, 300])
def test_verify_all_pairs(gkctx, max_len):
    rng = np.random.default_rng(max_len)
    ref = gen.c0_reference()
    gk.gk_load_reference(gkctx, ref)
    reads, off, pr, pos, e = edited_pairs(rng, ref, 6000, max_len=max_len)
    say(f"case: verify all, max_len={max_len}")
    d = verify(gkctx, reads, off, pr, pos, e, max_len)
    want = oracle_dist(ref, reads, off, pr, pos, e)
    bad = np.nonzero(d != want)[0]
    assert len(bad) == 0, (f"{len(bad)} differ; first {bad[0]}: gpu {d[bad[0]]} oracle "
                           f"{want[bad[0]]} e={e[bad[0]]} m={off[bad[0] + 1] - off[bad[0]]}")
    assert np.any(d <= e) and np.any(d == e.astype(np.uint16) + 1)


def test_verify_thresholds_and_lengths(gkctx):
    """Every e in 0..31 (the 32-bit band up to 15, the 64-bit band above) on
    lengths 1..40 and 500-512, and e > 31 gives GK_EST_NONE."""
    rng = np.random.default_rng(77)
    ref = gen.c0_reference()
    gk.gk_load_reference(gkctx, ref)
    reads, off, pr, pos, _ = edited_pairs(rng, ref, 4000, max_len=40)
    e = (np.arange(len(pos)) % 33).astype(np.uint8)
    say("case: verify thresholds 0..32, lengths 1..40")
    d = verify(gkctx, reads, off, pr, pos, e, 40)
    ok = e <= 31
    want = oracle_dist(ref, reads, off, pr[ok], pos[ok], e[ok])
    assert np.array_equal(d[ok], want)
    assert np.all(d[~ok] == gk.GK_EST_NONE)
    reads, off, pr, pos, e = edited_pairs(rng, ref, 300, max_len=512, min_len=500)
    say("case: verify lengths 500-512")
    d = verify(gkctx, reads, off, pr, pos, e, 512)
    want = oracle_dist(ref, reads, off, pr, pos, e)
    assert np.array_equal(d, want)


@pytest.mark.parametrize("m,e", [(100, 0), (100, 5), (37, 3), (100, 7), (256, 7), (250, 6),
                                 (400, 6), (100, 15), (150, 16), (250, 25), (512, 31),
                                 (300, 20)])
def test_verify_uniform_waves(gkctx, m, e):
    """One length and one threshold for the whole batch: every wave takes the
    path whose band shifts and trip counts are scalar (both band widths).
    Given as a per-pair array the pairs run one per lane; given as the batch's
    uniform e (<= 7, up to 256 bases) two pairs share a band word; longer
    reads with a uniform e <= 7 take the one-pair loop."""
    rng = np.random.default_rng(1000 + m + e)
    ref = gen.c0_reference()
    gk.gk_load_reference(gkctx, ref)
    reads, off, pr, pos, _ = edited_pairs(rng, ref, 3001, max_len=m, min_len=m)
    ev = np.full(len(pos), e, np.uint8)
    want = oracle_dist(ref, reads, off, pr, pos, ev)
    for form in ("per-pair", "uniform"):
        say(f"case: verify uniform m={m} e={e} ({form} e)")
        d = (verify(gkctx, reads, off, pr, pos, ev, m) if form == "per-pair" else
             verify(gkctx, reads, off, pr, pos, None, m, e_uniform=e))
        bad = np.nonzero(d != want)[0]
        assert len(bad) == 0, (f"{form}: {len(bad)} differ; first {bad[0]}: gpu {d[bad[0]]} "
                               f"oracle {want[bad[0]]}")
    assert np.any(want <= e) and np.any(want == e + 1)


@pytest.mark.parametrize("m,e", [(64, 0), (128, 3), (200, 7), (256, 5)])
def test_verify_paired_mixed_waves(gkctx, m, e):
    """A batch-wide e <= 7 on reads of up to 256 bases, with runs of one
    length, single odd lengths, gate failures (unknown base, empty read,
    window past the end, read index out of range) and random lengths cycling
    every 64 pairs.  The listing orders each group by length, so blocks of
    one length run two pairs per band word, and blocks that straddle two of
    the many short length runs are handed to the one-pair kernel; gate
    failures give GK_EST_NONE on either path."""
    rng = np.random.default_rng(5000 + m + e)
    ref = gen.c0_reference()
    gk.gk_load_reference(gkctx, ref)
    n = 6000
    reads, off, pr, pos, _ = edited_pairs(rng, ref, n, max_len=m, min_len=m)
    seqs = [reads[off[i]:off[i + 1]].tobytes() for i in range(n)]
    kind = (np.arange(n) // 64) % 4
    status = np.zeros(n, bool)
    for i in range(n):
        if kind[i] == 1 and i % 64 == 17:                  # one odd length in the wave
            seqs[i] = seqs[i][:m - 1 - int(rng.integers(0, min(m - 1, 9)))]
        elif kind[i] == 2 and i % 5 == 0:                  # gate failures among equals
            c = (i // 5) % 4
            status[i] = True
            if c == 0:
                s_ = bytearray(seqs[i])
                s_[int(rng.integers(0, m))] = ord("N")
                seqs[i] = bytes(s_)
            elif c == 1:
                seqs[i] = b""
            elif c == 2:
                pos[i] = len(ref) - m // 2
            else:
                pr[i] = n + 7
        elif kind[i] == 3:                                 # random lengths
            seqs[i] = seqs[i][:int(rng.integers(1, m + 1))]
    reads, off = concat_reads(seqs)
    ev = np.full(n, e, np.uint8)
    ok = ~status
    want = np.full(n, gk.GK_EST_NONE, np.uint16)
    want[ok] = oracle_dist(ref, reads, off, pr[ok], pos[ok], ev[ok])
    say(f"case: verify paired mixed waves m={m} e={e}")
    d = verify(gkctx, reads, off, pr, pos, None, m, e_uniform=e)
    bad = np.nonzero(d != want)[0]
    assert len(bad) == 0, (f"{len(bad)} differ; first {bad[0]} (kind {kind[bad[0]]}): gpu "
                           f"{d[bad[0]]} want {want[bad[0]]}")
    assert np.any(want[ok] <= e) and np.any(want == e + 1)


def test_verify_paired_deferral_at_scale(gkctx):
    """2^21 pairs of four read lengths (64-128 bp) with a batch-wide e = 4,
    every pair verified: each listing group is ordered by length, the paired
    kernel's persistent loop runs several steps per lane, and the blocks that
    straddle two lengths (in every group) go to the one-pair kernel through
    the deferred list.  Every distance is at most e + 1; a sample equals the
    oracle's."""
    ref = gen.c1_reference(20_000_000)
    gk.gk_load_reference(gkctx, ref)
    ps = gen.pairs(ref, seed=4242, n_reads=320_000, lengths=[64, 80, 100, 128],
                   cand_kind=gen.CAND_GEOM, cand_param=1 / 8, cand_cap=64, true_frac=0.5,
                   edit_kind=gen.EDIT_RATE, edit_param=1.2, e_value=4,
                   band_cands=True).take_pairs(1 << 21)
    n = ps.n_pairs
    assert n == 1 << 21
    say(f"case: verify paired deferral at scale, {n} pairs, e=4")
    d = verify(gkctx, ps.reads, ps.read_off, ps.pair_read, ps.cand_pos, None, 128, e_uniform=4)
    assert np.all(d <= 5)
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(n, size=1 << 14, replace=False))
    want = oracle.levenshtein_batch(ps.reads, ps.read_off, ref, ps.pair_read[idx],
                                    ps.cand_pos[idx], 4, n_threads=gen.default_threads())
    bad = np.nonzero(d[idx] != want)[0]
    assert len(bad) == 0, (f"{len(bad)} differ; first pair {idx[bad[0]]}: gpu "
                           f"{d[idx[bad[0]]]} oracle {want[bad[0]]}")
    assert np.any(want <= 4) and np.any(want == 5)


def test_verify_after_filter_and_status(gkctx):
    """Only GK_ACCEPT pairs are verified; rejected, undefined (unknown base,
    window past the end) and invalid pairs give GK_EST_NONE."""
    ref = gen.c1_reference(2_000_000)
    gk.gk_load_reference(gkctx, ref)
    ps = gen.c1_pairs(ref, 5, n_pairs=1 << 16)
    say("case: verify after filter, config 1 slice")
    dr = device.encode_reads(gkctx, ps.reads, ps.read_off, max_len=100)
    dp = device.upload_pairs(None, ps.cand_pos)
    b = device.batch_for(dr, dp, e_uniform=5, max_read_len=100)
    gk.gk_filter(gkctx, b, None)
    dist = torch.empty(ps.n_pairs, dtype=torch.int16, device="cuda")
    gk.gk_verify(gkctx, b, dp.accept, dist, None)
    torch.cuda.synchronize()
    a, _ = device.results(dp)
    d = dist.cpu().numpy().view(np.uint16)
    acc = a == gk.GK_ACCEPT
    assert np.all(d[~acc] == gk.GK_EST_NONE)
    want = oracle.levenshtein_batch(ps.reads, ps.read_off, ref, ps.pair_read[acc],
                                    ps.cand_pos[acc], 5, n_threads=gen.default_threads())
    assert np.array_equal(d[acc], want)
    # status cases through the all-pairs form
    seqs = [ref[10:110].tobytes(), b"ACGTN" * 20, b"", ref[500:600].tobytes()]
    reads, off = concat_reads(seqs)
    pr = np.array([0, 1, 2, 3, 9], np.uint32)
    pos = np.array([10, 0, 0, len(ref) - 50, 0], np.uint32)
    e = np.array([3, 3, 3, 3, 3], np.uint8)
    d = verify(gkctx, reads, off, pr, pos, e, 128)
    assert list(d) == [0] + [gk.GK_EST_NONE] * 4


@pytest.mark.parametrize("k,doff", [(1, 1), (3, 8), (16, 8)])
def test_verify_unaligned_buffers(gkctx, k, doff):
    """accept and dist at offsets that are not 16-byte aligned take the
    byte-wise select; an aligned offset takes the vector one.  Both list the
    same pairs: distances for the accepted, GK_EST_NONE for the rest, and
    nothing written outside dist."""
    ref = gen.c1_reference(2_000_000)
    gk.gk_load_reference(gkctx, ref)
    ps = gen.c1_pairs(ref, 5, n_pairs=(1 << 15) + 37)
    n = ps.n_pairs
    say(f"case: verify buffer offsets accept +{k} B, dist +{2 * doff} B")
    dr = device.encode_reads(gkctx, ps.reads, ps.read_off, max_len=100)
    dp = device.upload_pairs(None, ps.cand_pos)
    gk.gk_filter(gkctx, device.batch_for(dr, dp, e_uniform=5, max_read_len=100), None)
    dp2 = device.upload_pairs(ps.pair_read[k:], ps.cand_pos[k:])
    b2 = device.batch_for(dr, dp2, e_uniform=5, max_read_len=100)
    dist_full = torch.full((n + doff + 1,), 0x1234, dtype=torch.int16, device="cuda")
    acc_view = dp.accept[k:]
    dist_view = dist_full[doff:doff + n - k]
    gk.gk_verify(gkctx, b2, acc_view, dist_view, None)
    torch.cuda.synchronize()
    a, _ = device.results(dp)
    a = a[k:]
    full = dist_full.cpu().numpy().view(np.uint16)
    assert np.all(full[:doff] == 0x1234) and np.all(full[doff + n - k:] == 0x1234)
    d = full[doff:doff + n - k]
    acc = a == gk.GK_ACCEPT
    assert np.all(d[~acc] == gk.GK_EST_NONE)
    want = oracle.levenshtein_batch(ps.reads, ps.read_off, ref, ps.pair_read[k:][acc],
                                    ps.cand_pos[k:][acc], 5, n_threads=gen.default_threads())
    assert np.array_equal(d[acc], want)


def test_verify_errors(gkctx):
    """Call errors: a NULL dist, no reference, bad arguments; an empty batch
    is a no-op."""
    ref = gen.c0_reference()
    gk.gk_load_reference(gkctx, ref)
    reads, off = concat_reads([ref[10:110].tobytes()])
    dr = device.encode_reads(gkctx, reads, off, max_len=100)
    dp = device.upload_pairs(np.array([0], np.uint32), np.array([10], np.uint32))
    b = device.batch_for(dr, dp, e_uniform=2, max_read_len=100)
    with pytest.raises(gk.GkError) as ei:
        gk.gk_verify(gkctx, b, None, None, None)
    assert ei.value.status == gk.GK_EINVAL and "dist" in str(ei.value)
    dist = torch.empty(1, dtype=torch.int16, device="cuda")
    bad = device.batch_for(dr, dp, e_uniform=2, max_read_len=600)
    with pytest.raises(gk.GkError) as ei:
        gk.gk_verify(gkctx, bad, None, dist, None)
    assert ei.value.status == gk.GK_EINVAL
    ctx2 = gk.gk_create(0)
    try:
        with pytest.raises(gk.GkError) as ei:
            gk.gk_verify(ctx2, b, None, dist, None)
        assert ei.value.status == gk.GK_ENOREF
    finally:
        gk.gk_destroy(ctx2)
    b.n_pairs = 0
    gk.gk_verify(gkctx, b, None, None, None)      # empty: nothing to check
    b.n_pairs = 1
    gk.gk_verify(gkctx, b, None, dist, None)
    torch.cuda.synchronize()
    assert int(dist.cpu().numpy().view(np.uint16)[0]) == 0


def test_verify_interleaved_layout(gkctx):
    """The interleaved read layout gives the same distances."""
    rng = np.random.default_rng(91)
    ref = gen.c0_reference()
    gk.gk_load_reference(gkctx, ref)
    reads, off, pr, pos, e = edited_pairs(rng, ref, 3000, max_len=250)
    say("case: verify interleaved layout")
    d1 = verify(gkctx, reads, off, pr, pos, e, 250, layout=gk.GK_READS_INTERLEAVED)
    want = oracle_dist(ref, reads, off, pr, pos, e)
    assert np.array_equal(d1, want)


@pytest.mark.parametrize("identity", [False, True])
def test_verify_decoys_per_pair_e(gkctx, identity):
    """A per-pair e on reads of 40-300 bases: edited pairs (distances on both
    sides of e) and pairs at unrelated positions (distance above e, capped at
    e + 1), e over both band widths; reads from the row-major copy (pair_read
    given) and in place (pair i on read i); then a smaller batch on the same
    context buffers."""
    rng = np.random.default_rng(6464 + identity)
    ref = gen.c0_reference()
    gk.gk_load_reference(gkctx, ref)
    for n in (20000, 7000):
        reads, off, pr, pos, e = edited_pairs(rng, ref, n, max_len=300, min_len=40)
        lens = (off[1:] - off[:-1]).astype(np.int64)
        decoy = rng.random(n) < 0.5
        pos[decoy] = rng.integers(0, len(ref) - 300, int(decoy.sum())).astype(np.uint32)
        say(f"case: verify decoys per-pair e, identity={identity}, n={n}")
        d = verify(gkctx, reads, off, None if identity else pr, pos, e, 300)
        want = oracle_dist(ref, reads, off, pr, pos, e)
        bad = np.nonzero(d != want)[0]
        assert len(bad) == 0, (f"{len(bad)} differ; first {bad[0]}: gpu {d[bad[0]]} oracle "
                               f"{want[bad[0]]} e={e[bad[0]]} m={lens[bad[0]]}")
        long_ = lens > 64
        capped = d == e.astype(np.uint16) + 1
        assert np.sum(long_ & capped & decoy) > n // 10      # decoys: above e
        assert np.sum(long_ & ~capped) > n // 10              # within e

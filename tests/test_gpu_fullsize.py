"""Parity at the workloads' full sizes, in the launch configurations the
benchmark times: every pair against the oracle (directly at config 1, by a
digest of the oracle's outputs computed offline at configs 2 and 3, by
request at config 4), samples against the oracle pair by pair (which name the
first differing pair), and properties checked on every pair."""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_cases import assert_same, run_oracle, say
from paper_2103_14978_amd import device, gk

pytestmark = pytest.mark.gpu


def check_properties(a, s, e, m, label):
    """Every pair of an ACGT-only workload is ACCEPT or REJECT, with
    est <= m and accept iff est <= e."""
    assert set(np.unique(a)) <= {0, 1}, label
    assert np.all(s.astype(np.int64) <= m), label
    assert np.array_equal(a == 1, s.astype(np.int64) <= e), label


DIGESTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                       "fullsize_digests.json")


def digest_check(a, s, label):
    """Every pair: the SHA-256 of the outputs (accept codes, then estimates as
    little-endian uint16) equals the one tests/golden/make_fullsize_digests.py
    computed from the oracle on the same seeded workload."""
    with open(DIGESTS) as f:
        want = json.load(f)["points"][label]
    assert len(a) == want["n_pairs"], label
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(a, dtype="u1").tobytes())
    h.update(np.ascontiguousarray(s, dtype="<u2").tobytes())
    assert int((a == 1).sum()) == want["accepted"], f"{label}: accepted count"
    assert h.hexdigest() == want["sha256"], f"{label}: outputs differ from the oracle's"


def sample_check(ref, ps, a, s, e, k, seed, label):
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(ps.n_pairs, size=min(ps.n_pairs, k), replace=False))
    ee = e[idx] if isinstance(e, np.ndarray) else e
    ra, rs = run_oracle(ref, ps.reads, ps.read_off, ps.pair_read[idx], ps.cand_pos[idx], ee)
    assert_same(a[idx], s[idx], ra, rs, label)


def verify_check(ctx, ref, ps, b, dp, a, e, k, seed, label):
    """gk_verify after the filter, as the benchmark calls it: GK_EST_NONE on
    every pair the filter did not accept, at most e + 1 on every accepted
    one, and the oracle's capped edit distance on a sample of the accepted.
    e: one threshold, or one per pair."""
    dist = torch.empty(ps.n_pairs, dtype=torch.int16, device="cuda")
    gk.gk_verify(ctx, b, dp.accept, dist, None)
    torch.cuda.synchronize()
    d = dist.cpu().numpy().view(np.uint16)
    acc = a == gk.GK_ACCEPT
    ea = np.broadcast_to(np.asarray(e, np.int64), (ps.n_pairs,))
    assert np.all(d[~acc] == gk.GK_EST_NONE), label
    assert np.all(d[acc] <= ea[acc] + 1), label
    rng = np.random.default_rng(seed)
    idx = np.nonzero(acc)[0]
    idx = np.sort(rng.choice(idx, size=min(len(idx), k), replace=False))
    want = np.empty(len(idx), np.uint16)
    for v in np.unique(ea[idx]):
        sel = ea[idx] == v
        want[sel] = oracle.levenshtein_batch(ps.reads, ps.read_off, ref, ps.pair_read[idx[sel]],
                                             ps.cand_pos[idx[sel]], int(v),
                                             n_threads=gen.default_threads())
    bad = np.nonzero(d[idx] != want)[0]
    assert len(bad) == 0, (f"{label}: {len(bad)} of {len(idx)} differ; first pair "
                           f"{idx[bad[0]]}: gpu {d[idx[bad[0]]]} oracle {want[bad[0]]}")
    assert np.any(want <= ea[idx]), label
    return want


@pytest.fixture(scope="module")
def ref100m():
    return gen.c1_reference()


def test_config1_full(gkctx, ref100m):
    """2^24 pairs of 100 bp, e = 5, one candidate per read (pair_read NULL),
    split layout, automatic grid: the benchmark's launch, every pair against
    the oracle."""
    ref = ref100m
    gk.gk_load_reference(gkctx, ref)
    ps = gen.c1_pairs(ref, 5)
    say("case: config1 full 2^24 e=5")
    dr = device.encode_reads(gkctx, ps.reads, ps.read_off, max_len=100)
    dp = device.upload_pairs(None, ps.cand_pos)
    b = device.batch_for(dr, dp, e_uniform=5, max_read_len=100)
    gk.gk_filter(gkctx, b, None)
    torch.cuda.synchronize()
    a, s = device.results(dp)
    check_properties(a, s, 5, 100, "config1")
    ra, rs = run_oracle(ref, ps.reads, ps.read_off, ps.pair_read, ps.cand_pos, 5)
    assert_same(a, s, ra, rs, "config1 every pair")
    say("case: config1 full, reads encoded in the filter's launch (gk_filter_ascii)")
    d_ascii = torch.from_numpy(np.ascontiguousarray(ps.reads)).cuda()
    d_off = torch.from_numpy(ps.read_off.view(np.int64)).cuda()
    dp2 = device.upload_pairs(None, ps.cand_pos)
    dp2.accept.fill_(0xEE)
    b2 = gk.make_batch(n_reads=0, pitch=0, max_read_len=100, reads=None, read_len=None,
                       pair_read=None, cand_pos=dp2.cand_pos, accept=dp2.accept, est=dp2.est,
                       e_uniform=5)
    gk.gk_filter_ascii(gkctx, b2, d_ascii, d_off, None)
    torch.cuda.synchronize()
    a2, s2 = device.results(dp2)
    assert_same(a2, s2, ra, rs, "config1 fused, every pair")
    del d_ascii, d_off, dp2, b2, a2, s2
    say("case: config1 full verify of the accepted pairs")
    want = verify_check(gkctx, ref, ps, b, dp, a, 5, 1 << 15, 11, "config1 verify")
    assert np.any(want == 6)          # false accepts reach the cap


@pytest.mark.parametrize("m,es", [(150, (3, 7, 15)), (250, (5, 12, 25))])
def test_config2_full(gkctx, ref100m, m, es):
    """2^25 pairs at each (read length, e), several candidates per read:
    every pair against the oracle's digest."""
    ref = ref100m
    gk.gk_load_reference(gkctx, ref)
    for e in es:
        ps = gen.c2_pairs(ref, m, e)
        say(f"case: config2 full m={m} e={e} pairs={ps.n_pairs}")
        dr = device.encode_reads(gkctx, ps.reads, ps.read_off, max_len=m)
        dp = device.upload_pairs(ps.pair_read, ps.cand_pos)
        b = device.batch_for(dr, dp, e_uniform=e, max_read_len=m)
        gk.gk_filter(gkctx, b, None)
        torch.cuda.synchronize()
        a, s = device.results(dp)
        check_properties(a, s, e, m, f"config2 m={m} e={e}")
        sample_check(ref, ps, a, s, e, 1 << 13, e, f"config2 m={m} e={e}")
        digest_check(a, s, f"config2 m={m} e={e}")
        say(f"case: config2 full verify m={m} e={e}")
        verify_check(gkctx, ref, ps, b, dp, a, e, 1 << 13, 100 + e, f"config2 verify m={m} e={e}")
        del dr, dp, b


def test_config3_full(gkctx, ref100m):
    """2^26 mixed pairs: the autotuned persistent launch from its graph equals
    the plain launch and the oracle's digest on every pair."""
    ref = ref100m
    gk.gk_load_reference(gkctx, ref)
    ps = gen.c3_pairs(ref)
    say(f"case: config3 full pairs={ps.n_pairs}")
    dr = device.encode_reads(gkctx, ps.reads, ps.read_off, max_len=300)
    dp = device.upload_pairs(ps.pair_read, ps.cand_pos, ps.e)
    b = device.batch_for(dr, dp, max_read_len=300)
    gk.gk_tune_mixed(gkctx, b, None, sample_pairs=1 << 21)
    gk.gk_filter_mixed(gkctx, b, None)
    gk.gk_filter_mixed(gkctx, b, None)             # a graph replay
    torch.cuda.synchronize()
    a, s = device.results(dp)
    m = ps.read_len[ps.pair_read].astype(np.int64)
    check_properties(a, s, ps.e.astype(np.int64), m, "config3")
    dp2 = device.upload_pairs(ps.pair_read, ps.cand_pos, ps.e)
    gk.gk_filter(gkctx, device.batch_for(dr, dp2, max_read_len=300), None)
    torch.cuda.synchronize()
    a2, s2 = device.results(dp2)
    assert_same(a, s, a2, s2, "config3 mixed vs plain")
    sample_check(ref, ps, a, s, ps.e, 1 << 15, 3, "config3 sample")
    digest_check(a, s, "config3")
    say("case: config3 full verify of the accepted pairs")
    want = verify_check(gkctx, ref, ps, b, dp, a, ps.e, 1 << 15, 13, "config3 verify")
    assert np.any(want == 0)
    for opt, val in ((gk.GK_OPT_MIXED_TILE, 4096), (gk.GK_OPT_MIXED_PAIRS_PER_LANE, 1),
                     (gk.GK_OPT_MIXED_SORT_E, 1), (gk.GK_OPT_MIXED_BLOCKS_PER_CU, 0)):
        gk.gk_set_option(gkctx, opt, val)


def test_config4_full(gkctx):
    """3.1 Gbp resident reference; 16 requests of the served pool through the
    batched server, every pair against the oracle."""
    ref = gen.c4_reference()
    gk.gk_load_reference(gkctx, ref)
    reqs = [gen.c4_request(ref, k) for k in range(16)]
    say(f"case: config4 full, {sum(p.n_pairs for p in reqs)} pairs in 16 requests")
    srv = gk.gk_server_start(gkctx, 8 << 30, 64, 256, gk.GK_SERVER_BATCHED)
    try:
        objs = [gk.Request(p.reads, p.read_off, p.cand_pos, p.meta["e"], pair_read=p.pair_read)
                for p in reqs]
        tickets = [gk.gk_server_submit(srv, o) for o in objs]
        for t in tickets:
            st, _ = gk.gk_server_wait(srv, t, 120_000_000)
            assert st == gk.GK_OK
    finally:
        gk.gk_server_stop(srv)
    for k, (p, o) in enumerate(zip(reqs, objs)):
        ra, rs = run_oracle(ref, p.reads, p.read_off, p.pair_read, p.cand_pos, p.meta["e"])
        assert_same(o.accept, o.est, ra, rs, f"config4 request {k}")


def test_config4_2bit_reference(gkctx):
    """The 3.1 Gbp reference handed over as 2-bit words (several staging
    chunks, positions above 2^31) plus planted unknown-base runs: 16 requests'
    pairs through the plain launch, every pair against the oracle."""
    from gpu_cases import concat_reads, pack_2bit
    rng = np.random.default_rng(44)
    ref = gen.c4_reference()
    L = len(ref)
    starts = np.sort(rng.choice(L // 4096 - 2, 2000, replace=False)).astype(np.uint64) * 4096
    starts[-1] = L - 3000
    lens = rng.integers(1, 2000, len(starts)).astype(np.uint64)
    for s, l in zip(starts, lens):
        ref[int(s):int(s + l)] = ord("N")
    runs = np.stack([starts, lens], 1)
    reqs = [gen.c4_request(ref, k) for k in range(16)]
    # Send a quarter of each request's candidates next to a planted run.
    for p in reqs:
        k = p.n_pairs // 4
        near = starts[rng.integers(0, len(starts), k)].astype(np.int64) - rng.integers(0, 300, k)
        p.cand_pos[:k] = np.clip(near, 0, L - 300).astype(np.uint32)
    say(f"case: config4 2bit reference, {len(runs)} runs")
    gk.gk_load_reference_2bit(gkctx, pack_2bit(ref, gk.GK_READS_SPLIT, rng), L,
                              gk.GK_READS_SPLIT, runs)
    assert gk.gk_reference_info(gkctx) == (L, int(lens.sum()))
    for k, p in enumerate(reqs):
        m = int(p.meta["m"])
        dr = device.encode_reads(gkctx, p.reads, p.read_off, max_len=m)
        dp = device.upload_pairs(p.pair_read, p.cand_pos)
        gk.gk_filter(gkctx, device.batch_for(dr, dp, e_uniform=int(p.meta["e"]), max_read_len=m),
                     None)
        torch.cuda.synchronize()
        a, s = device.results(dp)
        ra, rs = run_oracle(ref, p.reads, p.read_off, p.pair_read, p.cand_pos, p.meta["e"])
        assert_same(a, s, ra, rs, f"config4 2bit request {k}")
        assert np.any(a == gk.GK_UNDEFINED)


def test_beyond_2e30_pairs(gkctx):
    """2^30 + 4133 pairs over 4096 reads: every entry point splits such a batch
    into launches of 2^30 pairs.  Plain launch against the oracle on the pairs
    around the split, the tail and a random sample; the mixed launch (with its
    accept bits) equal to the plain one on every pair; gk_verify on the
    sampled pairs against the oracle's distances."""
    import oracle
    n = (1 << 30) + 4133
    m, e, n_reads = 100, 5, 4096
    rng = np.random.default_rng(2030)
    ref = gen.c1_reference(20_000_000)
    gk.gk_load_reference(gkctx, ref)
    origins = rng.integers(8, len(ref) - m - 8, n_reads)
    seqs = []
    for o in origins:
        s = ref[o:o + m].copy()
        q = rng.integers(0, m, int(rng.integers(0, 8)))
        s[q] = np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, len(q))]
        seqs.append(s.tobytes())
    from gpu_cases import concat_reads
    reads, off = concat_reads(seqs)
    say(f"case: beyond 2^30, n_pairs={n}")
    pr = np.arange(n, dtype=np.uint32)
    np.remainder(pr, np.uint32(n_reads), out=pr)
    pos = rng.integers(0, len(ref) - m, n, dtype=np.uint32)
    step = 1 << 26
    for s0 in range(0, n, step):
        sl = slice(s0, min(n, s0 + step))
        idx = np.arange(sl.start, sl.stop, dtype=np.uint32)
        true = (idx % np.uint32(10)) < 3          # 30% of pairs at their read's origin
        pos[sl][true] = (origins[pr[sl][true]] + (idx[true] % 5).astype(np.int64) - 2).astype(
            np.uint32)
    dr = device.encode_reads(gkctx, reads, off, max_len=m)
    dp = device.upload_pairs(pr, pos, with_bits=True)
    b = device.batch_for(dr, dp, e_uniform=e, max_read_len=m)
    gk.gk_filter(gkctx, b, None)
    torch.cuda.synchronize()
    a, s = device.results(dp)
    # every pair is ACCEPT or REJECT, est <= m, accept iff est <= e
    assert int(a.max()) <= 1 and int(s.max()) <= m
    assert np.array_equal(a == 1, s <= e)
    split = 1 << 30
    idx = np.unique(np.concatenate([
        np.arange(split - 2048, split + 2048), np.arange(n - 600, n),
        rng.choice(n, 1 << 15, replace=False)]))
    ra, rs = run_oracle(ref, reads, off, pr[idx], pos[idx], e)
    assert_same(a[idx], s[idx], ra, rs, "beyond 2^30 plain sample")
    assert 0.2 < np.mean(a[idx] == 1) < 0.5
    for opt, val in ((gk.GK_OPT_MIXED_TILE, 4096), (gk.GK_OPT_MIXED_PAIRS_PER_LANE, 1),
                     (gk.GK_OPT_MIXED_SORT_E, 1), (gk.GK_OPT_MIXED_BLOCKS_PER_CU, 0)):
        gk.gk_set_option(gkctx, opt, val)
    dp.accept.fill_(0xEE)
    gk.gk_filter_mixed(gkctx, b, None)
    torch.cuda.synchronize()
    a2, s2 = device.results(dp)
    assert np.array_equal(a2, a) and np.array_equal(s2, s), "mixed differs from plain"
    del a2, s2
    bits = dp.accept_bits.cpu().numpy().view(np.uint8)
    got = np.unpackbits(bits[:(n + 7) // 8], bitorder="little")[:n]
    assert np.array_equal(got[idx].astype(bool), (a[idx] == 1) | (a[idx] == 2))
    del bits, got
    dist = torch.empty(n, dtype=torch.int16, device="cuda")
    gk.gk_verify(gkctx, b, dp.accept, dist, None)
    torch.cuda.synchronize()
    d = dist[torch.from_numpy(idx).cuda()].cpu().numpy().view(np.uint16)
    acc = a[idx] == gk.GK_ACCEPT
    assert np.all(d[~acc] == gk.GK_EST_NONE)
    want = oracle.levenshtein_batch(reads, off, ref, pr[idx][acc], pos[idx][acc], e,
                                    n_threads=gen.default_threads())
    assert np.array_equal(d[acc], want)
    del dist, dp, dr, b, pr, pos, a, s
    torch.cuda.empty_cache()


def test_beyond_2e30_identity(gkctx):
    """2^30 + 4133 pairs with no pair-to-read map (pair i uses read i) over
    4096 reads: the first 4096 pairs are compared, every other pair is
    GK_INVALID, also past the 2^30 split where each launch numbers its pairs
    from 0 again.  Plain and mixed launches and gk_verify (every pair)."""
    import oracle
    n = (1 << 30) + 4133
    m, e, n_reads = 100, 5, 4096
    rng = np.random.default_rng(2031)
    ref = gen.c1_reference(20_000_000)
    gk.gk_load_reference(gkctx, ref)
    origins = rng.integers(8, len(ref) - m - 8, n_reads)
    from gpu_cases import concat_reads
    reads, off = concat_reads([ref[o:o + m].tobytes() for o in origins])
    pos = rng.integers(0, len(ref) - m, n, dtype=np.uint32)
    pos[:n_reads:2] = origins[::2].astype(np.uint32)      # half of them at their origin
    say(f"case: beyond 2^30 identity, n_pairs={n}")
    dr = device.encode_reads(gkctx, reads, off, max_len=m)
    dp = device.upload_pairs(None, pos)
    b = device.batch_for(dr, dp, e_uniform=e, max_read_len=m)
    gk.gk_filter(gkctx, b, None)
    torch.cuda.synchronize()
    a, s = device.results(dp)
    pr = np.arange(n_reads, dtype=np.uint32)
    ra, rs = run_oracle(ref, reads, off, pr, pos[:n_reads], e)
    assert_same(a[:n_reads], s[:n_reads], ra, rs, "identity, pairs with a read")
    assert np.all(a[n_reads:] == gk.GK_INVALID), "pairs without a read"
    assert np.all(s[n_reads:] == gk.GK_EST_NONE)
    for opt, val in ((gk.GK_OPT_MIXED_TILE, 4096), (gk.GK_OPT_MIXED_PAIRS_PER_LANE, 1),
                     (gk.GK_OPT_MIXED_SORT_E, 1), (gk.GK_OPT_MIXED_BLOCKS_PER_CU, 0)):
        gk.gk_set_option(gkctx, opt, val)
    dp.accept.fill_(0xEE)
    gk.gk_filter_mixed(gkctx, b, None)
    torch.cuda.synchronize()
    a2, s2 = device.results(dp)
    assert np.array_equal(a2, a) and np.array_equal(s2, s), "mixed differs from plain"
    del a2, s2
    # The same pairs with their reads as text: reads past the 4096th are
    # empty (every later offset equals the text's end), so INVALID.
    say(f"case: beyond 2^30 identity, gk_filter_ascii, n_pairs={n}")
    d_ascii = torch.from_numpy(np.concatenate([reads, np.zeros(64, np.uint8)])).cuda()
    d_off = torch.full((n + 1,), int(off[-1]), dtype=torch.int64, device="cuda")
    d_off[:n_reads + 1] = torch.from_numpy(off.view(np.int64)).cuda()
    b3 = gk.make_batch(n_reads=0, pitch=0, max_read_len=m, reads=None, read_len=None,
                       pair_read=None, cand_pos=dp.cand_pos, accept=dp.accept, est=dp.est,
                       n_pairs=n, e_uniform=e)
    dp.accept.fill_(0xEE)
    gk.gk_filter_ascii(gkctx, b3, d_ascii, d_off, None)
    torch.cuda.synchronize()
    a3, s3 = device.results(dp)
    assert np.array_equal(a3, a) and np.array_equal(s3, s), "gk_filter_ascii differs from plain"
    del a3, s3, d_ascii, d_off, b3
    dist = torch.empty(n, dtype=torch.int16, device="cuda")
    gk.gk_verify(gkctx, b, None, dist, None)
    torch.cuda.synchronize()
    d = dist.cpu().numpy().view(np.uint16)
    want = oracle.levenshtein_batch(reads, off, ref, pr, pos[:n_reads], e,
                                    n_threads=gen.default_threads())
    assert np.array_equal(d[:n_reads], want)
    assert np.all(d[n_reads:] == gk.GK_EST_NONE)
    del dist, d, dp, dr, b, pos, a, s
    torch.cuda.empty_cache()

"""gk_filter_ascii: the filter that encodes its reads in the same launch
(pair i uses read i).  Bit-exact against the oracle and against
gk_encode_reads followed by gk_filter, accept bits included, on reads of
every length class the staging handles: many workgroups with a ragged last
one, reads of length 0, reads longer than max_read_len (INVALID), reads
longer than the rows hold (encoded from global memory), unknown bases and
lower case, per-pair and uniform e, the variant flags, and decreasing
offsets (an empty read)."""
import numpy as np
import pytest

import gen
from gpu_cases import assert_same, concat_reads, run_gpu, run_oracle, say
from paper_2103_14978_amd import device, gk

pytestmark = pytest.mark.gpu


def run_fused(ctx, reads, read_off, cand_pos, e, *, max_read_len, flags=0):
    """(accept, est, accept bits) of gk_filter_ascii; e is an int or a uint8
    array per pair."""
    import torch
    n = len(cand_pos)
    text = np.concatenate([np.asarray(reads, np.uint8), np.zeros(64, np.uint8)])
    d_ascii = torch.from_numpy(text).cuda()
    d_off = torch.from_numpy(np.asarray(read_off, np.uint64).view(np.int64)).cuda()
    per_pair = not np.isscalar(e) and not isinstance(e, int)
    dp = device.upload_pairs(None, cand_pos, e if per_pair else None, with_bits=True)
    dp.accept.fill_(0xEE)
    dp.est.fill_(0x5A5A)
    dp.accept_bits.fill_(-1)
    b = gk.make_batch(n_reads=0, pitch=0, max_read_len=max_read_len, reads=None,
                      read_len=None, pair_read=None, cand_pos=dp.cand_pos, accept=dp.accept,
                      est=dp.est, n_pairs=n, e=dp.e, e_uniform=0 if per_pair else int(e),
                      accept_bits=dp.accept_bits, flags=flags)
    gk.gk_filter_ascii(ctx, b, d_ascii, d_off, None)
    torch.cuda.synchronize()
    a, s = device.results(dp)
    return a, s, dp.accept_bits.cpu().numpy().view(np.uint64)


def _bits_of(a):
    want = (a == gk.GK_ACCEPT) | (a == gk.GK_UNDEFINED)
    return np.packbits(want, bitorder="little").view(np.uint8)


def test_fused_config1_against_plain_and_oracle(gkctx):
    """2^16 + 77 pairs of config 1 (100 bp, e = 5): equal to the two-launch
    path on every pair and to the oracle."""
    ref = gen.c1_reference(8_000_000)
    gk.gk_load_reference(gkctx, ref)
    ps = gen.c1_pairs(ref, 5, n_pairs=(1 << 16) + 77)
    say("case: fused config1 2^16+77")
    a, s, bits = run_fused(gkctx, ps.reads, ps.read_off, ps.cand_pos, 5, max_read_len=100)
    a2, s2, bits2 = run_gpu(gkctx, ref, ps.reads, ps.read_off, ps.pair_read, ps.cand_pos, 5,
                            max_read_len=100, with_bits=True, load_ref=False,
                            identity_as_null=True)
    assert_same(a, s, a2, s2, "fused vs encode + filter")
    nb = (len(a) + 63) // 64
    assert np.array_equal(bits[:nb], bits2[:nb]), "accept bits differ"
    ra, rs = run_oracle(ref, ps.reads, ps.read_off, ps.pair_read, ps.cand_pos, 5)
    assert_same(a, s, ra, rs, "fused vs oracle")


@pytest.mark.parametrize("max_len", [16, 100, 150, 300, 512])
def test_fused_lengths_unknown_bases_per_pair_e(gkctx, max_len):
    """Reads of every length from 0 to past max_read_len (and past what the
    rows hold), with unknown bases and lower case, e per pair."""
    rng = np.random.default_rng(4000 + max_len)
    ref = gen.c1_reference(4_000_000)
    gk.gk_load_reference(gkctx, ref)
    n = 3 * 256 + 113
    lens = rng.integers(0, max_len + 1, n)
    lens[::37] = max_len + rng.integers(1, 40, len(lens[::37]))    # INVALID, beyond the rows
    lens[5::41] = 0
    pos = rng.integers(0, len(ref) - 700, n).astype(np.uint32)
    seqs = []
    for i in range(n):
        m = int(lens[i])
        s = ref[pos[i]:pos[i] + m].copy()
        k = rng.integers(0, 4)
        if m and k:
            idx = rng.integers(0, m, k)
            s[idx] = rng.choice(np.frombuffer(b"ACGT", np.uint8), k)
        if m and i % 29 == 0:
            s[rng.integers(0, m)] = ord("N")
        if m and i % 31 == 0:
            s = np.char.lower(s.view("S1")).view(np.uint8)
        seqs.append(s.tobytes())
    reads, off = concat_reads(seqs)
    e = rng.integers(0, min(max_len // 8, 40) + 1, n).astype(np.uint8)
    say(f"case: fused lengths max_len={max_len} pairs={n}")
    a, s, bits = run_fused(gkctx, reads, off, pos, e, max_read_len=max_len)
    ra, rs = run_oracle(ref, reads, off, np.arange(n, dtype=np.uint32), pos, e)
    over = lens > max_len           # the launch's bound, below the oracle's own
    ra[over], rs[over] = gk.GK_INVALID, gk.GK_EST_NONE
    assert_same(a, s, ra, rs, f"fused vs oracle, max_len={max_len}")
    assert np.array_equal(bits.view(np.uint8)[:(n + 7) // 8], _bits_of(ra)[:(n + 7) // 8])
    assert np.any(ra == gk.GK_INVALID) and np.any(ra == gk.GK_UNDEFINED)


@pytest.mark.parametrize("flags", [gk.GK_FLAG_NO_REFINE, gk.GK_FLAG_HAMMING_FASTPATH])
def test_fused_variant_flags(gkctx, flags):
    """Variant semantics: equal to the two-launch path with the same flags."""
    ref = gen.c1_reference(4_000_000)
    gk.gk_load_reference(gkctx, ref)
    ps = gen.c1_pairs(ref, 4, n_pairs=5000)
    say(f"case: fused flags={flags}")
    a, s, _ = run_fused(gkctx, ps.reads, ps.read_off, ps.cand_pos, 4, max_read_len=100,
                        flags=flags)
    dr = device.encode_reads(gkctx, ps.reads, ps.read_off, max_len=100)
    dp = device.upload_pairs(None, ps.cand_pos)
    gk.gk_filter(gkctx, device.batch_for(dr, dp, e_uniform=4, max_read_len=100, flags=flags))
    import torch
    torch.cuda.synchronize()
    a2, s2 = device.results(dp)
    assert_same(a, s, a2, s2, f"fused vs encode + filter, flags={flags}")


def test_fused_decreasing_offsets_and_errors(gkctx):
    """An end offset below its start gives an empty read (INVALID), the other
    reads are unaffected; argument errors."""
    import torch
    ref = gen.c1_reference(2_000_000)
    gk.gk_load_reference(gkctx, ref)
    ps = gen.c1_pairs(ref, 3, n_pairs=600)
    off = ps.read_off.copy()
    off[300] = off[299] - 1 if off[299] > 0 else 0      # read 299 ends before it starts
    say("case: fused decreasing offset")
    a, s, _ = run_fused(gkctx, ps.reads, off, ps.cand_pos, 3, max_read_len=100)
    assert a[299] == gk.GK_INVALID and s[299] == gk.GK_EST_NONE
    ra, rs = run_oracle(ref, ps.reads, ps.read_off, ps.pair_read, ps.cand_pos, 3)
    good = np.ones(600, bool)
    good[[299, 300]] = False
    assert_same(a[good], s[good], ra[good], rs[good], "fused, other reads")
    # errors: pair_read given, NULL text, unaligned text
    d_ascii = torch.zeros(1024, dtype=torch.uint8, device="cuda")
    d_off = torch.zeros(601, dtype=torch.int64, device="cuda")
    dp = device.upload_pairs(np.arange(600), ps.cand_pos)
    b = gk.make_batch(n_reads=0, pitch=0, max_read_len=100, reads=None, read_len=None,
                      pair_read=dp.pair_read, cand_pos=dp.cand_pos, accept=dp.accept,
                      est=dp.est, n_pairs=600, e_uniform=3)
    for args in ((d_ascii, d_off), (None, d_off), (d_ascii[1:], d_off)):
        with pytest.raises(gk.GkError) as ei:
            gk.gk_filter_ascii(gkctx, b, *args)
        assert ei.value.status == gk.GK_EINVAL
        b.pair_read = None
    b.n_pairs = 0
    gk.gk_filter_ascii(gkctx, b, d_ascii, d_off)

"""gk_filter_mixed_noalloc, the entry point that allocates nothing (its
scratch is a fixed device array of the library), against gk_filter_mixed
and the oracle, element by element, on two calls in a row with the second
one smaller.  The batches hold pairs with more than 31 shifts, so the
residual list in the fixed array is used, and a ragged tail."""
import numpy as np
import pytest

import gen
from gpu_cases import assert_same, run_oracle, say
from paper_2103_14978_amd import device, gk

pytestmark = pytest.mark.gpu

MAX_LEN = 400


def _pairs(seed, n_reads):
    # 200 / 300 / 400 bp reads, per-pair e up to 12 % of the length (up to
    # 48 shifts: pairs with more than 31 go to the residual pass)
    ref = gen.c1_reference(8_000_000)
    ps = gen.pairs(ref, seed=seed, n_reads=n_reads, lengths=[200, 300, 400],
                   cand_kind=gen.CAND_GEOM, cand_param=1 / 4, cand_cap=16, true_frac=0.5,
                   edit_kind=gen.EDIT_RATE, edit_param=1.2, e_frac=0.12, band_cands=True)
    return ref, ps


def _filter_both(ctx, ps):
    import torch
    dr = device.encode_reads(ctx, ps.reads, ps.read_off, max_len=MAX_LEN)
    dp_m = device.upload_pairs(ps.pair_read, ps.cand_pos, ps.e, with_bits=True)
    dp_n = device.upload_pairs(ps.pair_read, ps.cand_pos, ps.e, with_bits=True)
    for dp in (dp_m, dp_n):
        dp.accept.fill_(0xEE)
        dp.est.fill_(0x5A5A)
        dp.accept_bits.fill_(-1)
    torch.cuda.synchronize()
    gk.gk_filter_mixed(ctx, device.batch_for(dr, dp_m, max_read_len=MAX_LEN), None)
    torch.cuda.synchronize()
    gk.gk_filter_mixed_noalloc(ctx, device.batch_for(dr, dp_n, max_read_len=MAX_LEN), None)
    torch.cuda.synchronize()
    am, sm = device.results(dp_m)
    an, sn = device.results(dp_n)
    bm = dp_m.accept_bits.cpu().numpy()
    bn = dp_n.accept_bits.cpu().numpy()
    return (am, sm, bm), (an, sn, bn)


def test_noalloc_matches_mixed_on_two_calls(gkctx):
    ref, big = _pairs(5151, 24_000)
    _, small = _pairs(5152, 3_000)
    assert big.n_pairs > small.n_pairs > 0
    assert big.n_pairs <= gk.GK_NOALLOC_MAX_PAIRS
    kmax = np.minimum(big.e.astype(np.int64), big.read_len[big.pair_read].astype(np.int64) - 1)
    assert np.sum(kmax > 31) > 1000, "the batch must exercise the residual list"
    gk.gk_load_reference(gkctx, ref)
    for label, ps in (("first call", big), ("second call, smaller", small)):
        say(f"case: noalloc vs mixed, {label}, {ps.n_pairs} pairs")
        (am, sm, bm), (an, sn, bn) = _filter_both(gkctx, ps)
        assert_same(an, sn, am, sm, f"noalloc vs mixed, {label}")
        assert np.array_equal(bn, bm), f"accept bits differ, {label}"
        ra, rs = run_oracle(ref, ps.reads, ps.read_off, ps.pair_read, ps.cand_pos, ps.e)
        assert_same(an, sn, ra, rs, f"noalloc vs oracle, {label}")


def test_noalloc_limits(gkctx):
    """Beyond GK_NOALLOC_MAX_PAIRS: GK_ERANGE before anything is launched
    (the host check; the pair buffers are never read).  Empty batch: OK."""
    ref, ps = _pairs(5153, 200)
    gk.gk_load_reference(gkctx, ref)
    dr = device.encode_reads(gkctx, ps.reads, ps.read_off, max_len=MAX_LEN)
    dp = device.upload_pairs(ps.pair_read, ps.cand_pos, ps.e)
    b = device.batch_for(dr, dp, max_read_len=MAX_LEN)
    b.n_pairs = gk.GK_NOALLOC_MAX_PAIRS + 1
    with pytest.raises(gk.GkError) as ei:
        gk.gk_filter_mixed_noalloc(gkctx, b, None)
    assert ei.value.status == gk.GK_ERANGE
    b.n_pairs = 0
    gk.gk_filter_mixed_noalloc(gkctx, b, None)

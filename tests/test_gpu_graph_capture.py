"""Library launches recorded into a caller's HIP graph: gk_filter,
gk_filter_ascii and gk_filter_mixed_noalloc (the entry point that allocates
nothing, for callers under graph capture) captured on a torch graph stream, then replayed several
times with the outputs cleared eagerly between replays.  Every replay equals
the eager launch of the same batches and the oracle, element by element.
The mixed batch holds pairs with more than 31 shifts, so the captured
sequence includes the residual pass over the fixed scratch array."""
import numpy as np
import pytest

import gen
from gpu_cases import assert_same, run_oracle, say
from paper_2103_14978_amd import device, gk

pytestmark = pytest.mark.gpu

MAX_LEN = 300


def _mixed_pairs(ref):
    return gen.pairs(ref, seed=7373, n_reads=6_000, lengths=[150, 250, 300],
                     cand_kind=gen.CAND_GEOM, cand_param=1 / 4, cand_cap=16, true_frac=0.5,
                     edit_kind=gen.EDIT_RATE, edit_param=1.2, e_frac=0.12, band_cands=True)


def test_capture_and_replay(gkctx):
    import torch
    ref = gen.c1_reference(8_000_000)
    gk.gk_load_reference(gkctx, ref)
    mixed = _mixed_pairs(ref)
    kmax = np.minimum(mixed.e.astype(np.int64),
                      mixed.read_len[mixed.pair_read].astype(np.int64) - 1)
    assert np.sum(kmax > 31) > 100, "the batch must exercise the residual pass"
    plain = gen.c1_pairs(ref, 4, n_pairs=(1 << 15) + 41)

    dr_m = device.encode_reads(gkctx, mixed.reads, mixed.read_off, max_len=MAX_LEN)
    dp_m = device.upload_pairs(mixed.pair_read, mixed.cand_pos, mixed.e, with_bits=True)
    b_m = device.batch_for(dr_m, dp_m, max_read_len=MAX_LEN)
    dr_p = device.encode_reads(gkctx, plain.reads, plain.read_off, max_len=100)
    dp_p = device.upload_pairs(None, plain.cand_pos, with_bits=True)
    b_p = device.batch_for(dr_p, dp_p, e_uniform=4, max_read_len=100)
    # the same pairs with their reads as text, encoded in the filter's launch
    d_ascii = torch.from_numpy(np.concatenate([plain.reads, np.zeros(64, np.uint8)])).cuda()
    d_off = torch.from_numpy(plain.read_off.view(np.int64)).cuda()
    dp_a = device.upload_pairs(None, plain.cand_pos, with_bits=True)
    b_a = gk.make_batch(n_reads=0, pitch=0, max_read_len=100, reads=None, read_len=None,
                        pair_read=None, cand_pos=dp_a.cand_pos, accept=dp_a.accept,
                        est=dp_a.est, e_uniform=4, accept_bits=dp_a.accept_bits)
    torch.cuda.synchronize()

    # eager launches: the expected bytes
    gk.gk_filter_mixed_noalloc(gkctx, b_m, None)
    gk.gk_filter(gkctx, b_p, None)
    gk.gk_filter_ascii(gkctx, b_a, d_ascii, d_off, None)
    torch.cuda.synchronize()
    want_m = device.results(dp_m) + (dp_m.accept_bits.cpu().numpy(),)
    want_p = device.results(dp_p) + (dp_p.accept_bits.cpu().numpy(),)
    got_a = device.results(dp_a) + (dp_a.accept_bits.cpu().numpy(),)
    assert_same(got_a[0], got_a[1], want_p[0], want_p[1], "eager ascii vs plain")
    assert np.array_equal(got_a[2], want_p[2]), "eager ascii accept bits"
    ra, rs = run_oracle(ref, mixed.reads, mixed.read_off, mixed.pair_read, mixed.cand_pos,
                        mixed.e)
    assert_same(want_m[0], want_m[1], ra, rs, "eager noalloc vs oracle")
    ra, rs = run_oracle(ref, plain.reads, plain.read_off, plain.pair_read, plain.cand_pos, 4)
    assert_same(want_p[0], want_p[1], ra, rs, "eager plain vs oracle")

    def clear():
        for dp in (dp_m, dp_p, dp_a):
            dp.accept.fill_(0xEE)
            dp.est.fill_(0x5A5A)
            dp.accept_bits.fill_(-1)

    say("case: graph capture of gk_filter_mixed_noalloc + gk_filter + gk_filter_ascii")
    clear()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        s = torch.cuda.current_stream()
        gk.gk_filter_mixed_noalloc(gkctx, b_m, s)
        gk.gk_filter(gkctx, b_p, s)
        gk.gk_filter_ascii(gkctx, b_a, d_ascii, d_off, s)
    torch.cuda.synchronize()
    for rep in range(4):
        clear()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got_m = device.results(dp_m) + (dp_m.accept_bits.cpu().numpy(),)
        got_p = device.results(dp_p) + (dp_p.accept_bits.cpu().numpy(),)
        assert_same(got_m[0], got_m[1], want_m[0], want_m[1], f"replay {rep}: noalloc")
        assert np.array_equal(got_m[2], want_m[2]), f"replay {rep}: noalloc accept bits"
        assert_same(got_p[0], got_p[1], want_p[0], want_p[1], f"replay {rep}: plain")
        assert np.array_equal(got_p[2], want_p[2]), f"replay {rep}: plain accept bits"
        got_a = device.results(dp_a) + (dp_a.accept_bits.cpu().numpy(),)
        assert_same(got_a[0], got_a[1], want_p[0], want_p[1], f"replay {rep}: ascii")
        assert np.array_equal(got_a[2], want_p[2]), f"replay {rep}: ascii accept bits"
        # eager work between replays, on the same scratch array
        gk.gk_filter_mixed_noalloc(gkctx, b_m, None)
        torch.cuda.synchronize()
    del g

"""The serving loop (gk_server_*): continuous batching must not change a
single byte.  Each request's results alone equal its results in the mix
(tolerance: bit-identical) and the oracle's; the sequential per-request mode
gives the same bytes; admission limits queue requests instead of failing."""
import ctypes

import numpy as np
import pytest

import gen
from gpu_cases import assert_same, run_oracle, say
from paper_2103_14978_amd import gk

pytestmark = pytest.mark.gpu


def make_requests(ref, count, seed, max_pairs=30_000):
    reqs = []
    rng = np.random.default_rng(seed)
    for k in range(count):
        n = int(np.exp(rng.uniform(np.log(50), np.log(max_pairs))))
        m = int(rng.integers(100, 251))
        e = int(rng.integers(0, m // 10 + 1))
        ps = gen.pairs(ref, seed=seed * 1000 + k, n_reads=n // 8 + 8, lengths=[m],
                       cand_kind=gen.CAND_GEOM, cand_param=1 / 8, cand_cap=64, true_frac=0.45,
                       edit_kind=gen.EDIT_RATE, edit_param=1.2, decoy_kind=gen.DECOY_SEEDS,
                       seed_k=16, e_value=e, band_cands=True).take_pairs(n)
        reqs.append((ps, e))
    return reqs


def run_server(ctx, reqs, *, mode=gk.GK_SERVER_BATCHED, budget=1 << 30, slots=64, alone=False):
    srv = gk.gk_server_start(ctx, budget, slots, 256, mode)
    outs = []
    try:
        objs = [gk.Request(ps.reads, ps.read_off, ps.cand_pos, e, pair_read=ps.pair_read)
                for ps, e in reqs]
        if alone:
            for o in objs:
                t = gk.gk_server_submit(srv, o)
                st, stats = gk.gk_server_wait(srv, t, 60_000_000)
                assert st == gk.GK_OK
        else:
            tickets = [gk.gk_server_submit(srv, o) for o in objs]
            for t in tickets:
                st, stats = gk.gk_server_wait(srv, t, 60_000_000)
                assert st == gk.GK_OK
                assert stats.t_done_us >= stats.t_admit_us >= stats.t_submit_us
        outs = [(o.accept.copy(), o.est.copy()) for o in objs]
        counters = gk.gk_server_counters(srv)
    finally:
        gk.gk_server_stop(srv)
    return outs, counters


@pytest.fixture(scope="module")
def served(gkctx):
    ref = gen.c1_reference(20_000_000)
    reqs = make_requests(ref, 40, 91)
    want = [run_oracle(ref, ps.reads, ps.read_off, ps.pair_read, ps.cand_pos, e)
            for ps, e in reqs]
    return ref, reqs, want


def test_alone_equals_mix_equals_oracle(gkctx, served):
    ref, reqs, want = served
    gk.gk_load_reference(gkctx, ref)
    say("case: serve alone")
    alone, _ = run_server(gkctx, reqs, alone=True)
    say("case: serve mixed")
    mixed, (ticks, max_per_tick, pairs) = run_server(gkctx, reqs)
    assert pairs == sum(ps.n_pairs for ps, _ in reqs)
    for k, ((aa, sa), (am, sm), (ra, rs)) in enumerate(zip(alone, mixed, want)):
        assert_same(am, sm, aa, sa, f"request {k}: mix vs alone")
        assert_same(am, sm, ra, rs, f"request {k}: vs oracle")
    print(f"ticks={ticks} max requests in one tick={max_per_tick}")


def test_sequential_mode_same_bytes(gkctx, served):
    ref, reqs, want = served
    gk.gk_load_reference(gkctx, ref)
    say("case: serve sequential")
    seq, _ = run_server(gkctx, reqs, mode=gk.GK_SERVER_SEQUENTIAL)
    for k, ((a, s), (ra, rs)) in enumerate(zip(seq, want)):
        assert_same(a, s, ra, rs, f"sequential request {k}")


def test_tiny_budget_and_slots_queue(gkctx, served):
    ref, reqs, want = served
    gk.gk_load_reference(gkctx, ref)
    say("case: serve tiny budget")
    big = max(ps.n_pairs for ps, _ in reqs)
    # room for roughly one large request at a time, two slots
    outs, _ = run_server(gkctx, reqs, budget=max(1 << 20, big * 64), slots=2)
    for k, ((a, s), (ra, rs)) in enumerate(zip(outs, want)):
        assert_same(a, s, ra, rs, f"tiny budget request {k}")


SERVER_DEFAULTS = {gk.GK_OPT_SERVER_PART_PAIRS: 1 << 17, gk.GK_OPT_SERVER_TICK_PAIRS: 1 << 20,
                   gk.GK_OPT_MIXED_TILE: 4096, gk.GK_OPT_MIXED_PAIRS_PER_LANE: 1,
                   gk.GK_OPT_MIXED_SORT_E: 1, gk.GK_OPT_MIXED_BLOCKS_PER_CU: 0,
                   gk.GK_OPT_SERVER_COPY_STREAMS: 4}


def with_options(ctx, opts, fn):
    for k, v in opts.items():
        gk.gk_set_option(ctx, k, v)
    try:
        return fn()
    finally:
        for k in opts:
            gk.gk_set_option(ctx, k, SERVER_DEFAULTS[k])


@pytest.mark.parametrize("part,tick,tile,ppl", [(256, 4096, 2048, 1), (3000, 20_000, 8192, 2),
                                                (1 << 17, 1 << 20, 4096, 2)])
def test_requests_split_over_ticks(gkctx, served, part, tick, tile, ppl):
    """Requests spread over several ticks in parts (one tick holding parts
    of several requests), under several tick tunings: every request's bytes
    equal the oracle's."""
    ref, reqs, want = served
    gk.gk_load_reference(gkctx, ref)
    say(f"case: serve split part={part} tick={tick} tile={tile} ppl={ppl}")
    opts = {gk.GK_OPT_SERVER_PART_PAIRS: part, gk.GK_OPT_SERVER_TICK_PAIRS: tick,
            gk.GK_OPT_MIXED_TILE: tile, gk.GK_OPT_MIXED_PAIRS_PER_LANE: ppl}
    outs, (ticks, max_parts, pairs) = with_options(gkctx, opts, lambda: run_server(gkctx, reqs))
    total = sum(ps.n_pairs for ps, _ in reqs)
    assert pairs == total
    assert ticks >= total // tick
    for k, ((a, s), (ra, rs)) in enumerate(zip(outs, want)):
        assert_same(a, s, ra, rs, f"split request {k}")


@pytest.mark.parametrize("streams", [1, 2, 3])
def test_copy_streams(gkctx, served, streams):
    """The loader taking 1, 2 or 3 copy streams in turn (4 is the default),
    with requests split over ticks: every request's bytes equal the
    oracle's."""
    ref, reqs, want = served
    gk.gk_load_reference(gkctx, ref)
    say(f"case: serve copy streams={streams}")
    opts = {gk.GK_OPT_SERVER_COPY_STREAMS: streams, gk.GK_OPT_SERVER_PART_PAIRS: 3000,
            gk.GK_OPT_SERVER_TICK_PAIRS: 20_000}
    outs, (ticks, max_parts, pairs) = with_options(gkctx, opts, lambda: run_server(gkctx, reqs))
    assert pairs == sum(ps.n_pairs for ps, _ in reqs)
    for k, ((a, s), (ra, rs)) in enumerate(zip(outs, want)):
        assert_same(a, s, ra, rs, f"copy streams {streams} request {k}")


def test_split_requests_one_candidate_per_read(gkctx, served):
    """Requests with no pair_read (pair i uses read i) split into parts: each
    part's reads are found at the part's offset."""
    ref = served[0]
    gk.gk_load_reference(gkctx, ref)
    reqs = []
    for k, (n, m, e) in enumerate([(9000, 100, 3), (700, 150, 7), (20_000, 250, 12)]):
        ps = gen.pairs(ref, seed=777 + k, n_reads=n, lengths=[m], true_frac=0.5,
                       edit_kind=gen.EDIT_RATE, edit_param=1.2, e_value=e)
        assert np.array_equal(ps.pair_read, np.arange(n))
        reqs.append((ps, e))
    say("case: serve split, one candidate per read")
    opts = {gk.GK_OPT_SERVER_PART_PAIRS: 1000, gk.GK_OPT_SERVER_TICK_PAIRS: 4096}

    def go():
        srv = gk.gk_server_start(gkctx, 1 << 28, 16, 256, gk.GK_SERVER_BATCHED)
        try:
            objs = [gk.Request(ps.reads, ps.read_off, ps.cand_pos, e) for ps, e in reqs]
            for t in [gk.gk_server_submit(srv, o) for o in objs]:
                assert gk.gk_server_wait(srv, t, 60_000_000)[0] == gk.GK_OK
            return objs
        finally:
            gk.gk_server_stop(srv)
    objs = with_options(gkctx, opts, go)
    for k, (o, (ps, e)) in enumerate(zip(objs, reqs)):
        ra, rs = run_oracle(ref, ps.reads, ps.read_off, ps.pair_read, ps.cand_pos, e)
        assert_same(o.accept, o.est, ra, rs, f"identity request {k}")


def test_limits_timeout_and_empty(gkctx, served):
    ref, reqs, want = served
    gk.gk_load_reference(gkctx, ref)
    srv = gk.gk_server_start(gkctx, 1 << 20, 4, 150, gk.GK_SERVER_BATCHED)
    try:
        ps, e = max(reqs, key=lambda r: r[0].n_pairs)
        # a read longer than the server's max_read_len
        long_read = gk.Request(np.frombuffer(b"A" * 200, np.uint8), np.array([0, 200]),
                               np.array([0], np.uint32), 1)
        with pytest.raises(gk.GkError) as ei:
            gk.gk_server_submit(srv, long_read)
        assert ei.value.status == gk.GK_ERANGE
        # a request larger than the whole budget
        n = 200_000
        big = gk.Request(np.frombuffer(b"ACGT" * 25, np.uint8), np.array([0, 100]),
                         np.zeros(n, np.uint32), 1, pair_read=np.zeros(n, np.uint32))
        with pytest.raises(gk.GkError) as ei:
            gk.gk_server_submit(srv, big)
        assert ei.value.status == gk.GK_ERANGE
        # empty request completes at once
        empty = gk.Request(np.zeros(0, np.uint8), np.array([0]), np.zeros(0, np.uint32), 1)
        t = gk.gk_server_submit(srv, empty)
        st, stats = gk.gk_server_wait(srv, t, 0)
        assert st == gk.GK_OK and stats.n_pairs == 0
        # timeout, then a real wait
        n = 20_000
        reads = np.frombuffer(ref[1000:1000 + 100].tobytes() * 10, np.uint8)
        req = gk.Request(reads, np.arange(0, 1001, 100), np.full(n, 1000, np.uint32), 2,
                         pair_read=np.arange(n, dtype=np.uint32) % 10)
        t = gk.gk_server_submit(srv, req)
        st, _ = gk.gk_server_wait(srv, t, 0)
        assert st in (gk.GK_ETIMEOUT, gk.GK_OK)
        if st == gk.GK_ETIMEOUT:
            st, _ = gk.gk_server_wait(srv, t, 60_000_000)
        assert st == gk.GK_OK
        assert np.all(req.accept == 1) and np.all(req.est == 0)
        assert gk.gk_server_wait(srv, 999_999, 0)[0] == gk.GK_EINVAL
    finally:
        gk.gk_server_stop(srv)


def test_unknown_bases_in_requests(gkctx):
    rng = np.random.default_rng(4)
    ref = bytearray(rng.choice(np.frombuffer(b"ACGT", np.uint8), 200_000).tobytes())
    for p in rng.integers(0, len(ref), 50):
        ref[int(p)] = ord("N")
    ref = np.frombuffer(bytes(ref), np.uint8).copy()
    gk.gk_load_reference(gkctx, ref)
    reqs = make_requests(ref, 6, 17, max_pairs=5000)
    for ps, _ in reqs[:3]:
        ps.reads[::997] = ord("N")
    say("case: serve unknown bases")
    outs, _ = run_server(gkctx, reqs)
    for k, ((a, s), (ps, e)) in enumerate(zip(outs, reqs)):
        ra, rs = run_oracle(ref, ps.reads, ps.read_off, ps.pair_read, ps.cand_pos, e)
        assert_same(a, s, ra, rs, f"unknown-base request {k}")


def test_stop_cancels_unadmitted(gkctx, served):
    """Stopping a busy sequential server returns once the admitted request is
    done; requests still queued are cancelled, not run."""
    import time
    ref, reqs, want = served
    gk.gk_load_reference(gkctx, ref)
    srv = gk.gk_server_start(gkctx, 1 << 30, 4, 256, gk.GK_SERVER_SEQUENTIAL)
    objs = [gk.Request(ps.reads, ps.read_off, ps.cand_pos, e, pair_read=ps.pair_read)
            for ps, e in reqs * 5]
    for o in objs:
        gk.gk_server_submit(srv, o)
    t = time.time()
    gk.gk_server_stop(srv)
    assert time.time() - t < 30


@pytest.mark.parametrize("mode,load_at,tick_at", [(gk.GK_SERVER_BATCHED, 12, 0),
                                                  (gk.GK_SERVER_BATCHED, 0, 2),
                                                  (gk.GK_SERVER_SEQUENTIAL, 5, 0)])
def test_injected_failure_ends_every_wait(gkctx, served, mode, load_at, tick_at):
    """A HIP call inside the server that reports an error (injected on the
    host: every kernel runs normally) ends the server's work without leaving
    a wait behind: every wait returns, GK_OK with the oracle's results for
    requests done before the failure and GK_EDEVICE for the rest; later
    submissions are refused and stop reports GK_EDEVICE."""
    ref, reqs, want = served
    gk.gk_load_reference(gkctx, ref)
    say(f"case: server injected failure mode={mode} load_at={load_at} tick_at={tick_at}")
    srv = gk.gk_server_start(gkctx, 1 << 30, 64, 256, mode)
    inject = gk.lib().gk_detail_server_inject_failure
    inject.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64]
    inject.restype = ctypes.c_int
    stopped = False
    try:
        assert inject(srv, load_at, tick_at) == gk.GK_OK
        objs = [gk.Request(ps.reads, ps.read_off, ps.cand_pos, e, pair_read=ps.pair_read)
                for ps, e in reqs]
        tickets = []
        for o in objs:
            try:
                tickets.append(gk.gk_server_submit(srv, o))
            except gk.GkError as err:            # the failure came first
                assert err.status == gk.GK_EDEVICE
                break
        statuses = []
        for k, t in enumerate(tickets):
            st, _ = gk.gk_server_wait(srv, t, 60_000_000)
            assert st in (gk.GK_OK, gk.GK_EDEVICE), st
            statuses.append(st)
            if st == gk.GK_OK:
                assert_same(objs[k].accept, objs[k].est, *want[k], f"request {k}")
        assert gk.GK_EDEVICE in statuses
        with pytest.raises(gk.GkError) as ei:
            gk.gk_server_submit(srv, objs[0])
        assert ei.value.status == gk.GK_EDEVICE
        stopped = True
        with pytest.raises(gk.GkError) as ei:
            gk.gk_server_stop(srv)
        assert ei.value.status == gk.GK_EDEVICE
    finally:
        if not stopped:
            try:
                gk.gk_server_stop(srv)
            except gk.GkError:
                pass

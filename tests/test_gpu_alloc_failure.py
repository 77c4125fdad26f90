"""Allocation failures: every entry point that allocates device or pinned host
memory returns GK_ENOMEM when one of its allocations fails, and the context
(or, for gk_create, the library) stays usable: the same call succeeds once
the failure is lifted, and a filter run afterwards equals the oracle.

The failure is injected by the library's test hook gk_detail_fail_alloc(n),
which makes the n-th allocation from then on report out-of-memory without
allocating; n runs over every allocation the call makes, so each error path
is taken once.  Nothing on the device fails: no kernel is launched with a
missing buffer."""
import ctypes

import numpy as np
import pytest

import gen
import oracle
from gpu_cases import assert_same, pack_2bit, say, unknown_runs
from paper_2103_14978_amd import device, gk

pytestmark = pytest.mark.gpu

E = 2
MAX_CALLS = 40          # more allocations than any single call makes


def _hook():
    f = gk.lib().gk_detail_fail_alloc
    f.argtypes = [ctypes.c_uint64]
    f.restype = ctypes.c_int
    return f


@pytest.fixture(scope="module")
def data():
    ref = gen.c0_reference()
    ps = gen.c0_pairs(ref, n_reads=3000)
    ra, rs = oracle.filter_batch(ps.reads, ps.read_off, ref, ps.pair_read, ps.cand_pos, E,
                                 n_threads=8)
    return ref, ps, ra, rs


def _filter_ok(ctx, data, load=True):
    """The context filters the config-0 pairs bit-exactly."""
    import torch
    ref, ps, ra, rs = data
    if load:
        gk.gk_load_reference(ctx, ref)
    dr = device.encode_reads(ctx, ps.reads, ps.read_off, max_len=100)
    dp = device.upload_pairs(ps.pair_read, ps.cand_pos)
    gk.gk_filter(ctx, device.batch_for(dr, dp, e_uniform=E, max_read_len=100), None)
    torch.cuda.synchronize()
    a, s = device.results(dp)
    assert_same(a, s, ra, rs, "filter after an allocation failure")


def _each_failure(make_ctx, call, after, label):
    """For n = 1, 2, ...: a fresh context, the n-th allocation of `call`
    fails -> GK_ENOMEM; then `call` again without the failure succeeds and
    `after` checks the context.  Stops at the first n past the call's last
    allocation (the call succeeds with the failure still pending)."""
    fail_at = _hook()
    seen = 0
    for n in range(1, MAX_CALLS + 1):
        say(f"case: alloc failure {label} n={n}")
        ctx = make_ctx()
        try:
            fail_at(n)
            try:
                call(ctx)
                status = gk.GK_OK
            except gk.GkError as ex:
                status = ex.status
            fail_at(0)
            if status == gk.GK_OK:
                break
            assert status == gk.GK_ENOMEM, f"{label}: allocation {n} failed with {status}"
            seen += 1
            call(ctx)
            after(ctx)
        finally:
            fail_at(0)
            gk.gk_destroy(ctx)
    else:
        raise AssertionError(f"{label}: still failing after {MAX_CALLS} allocations")
    assert seen >= 1, f"{label}: the call made no allocation"
    return seen


def test_create(data):
    fail_at = _hook()
    say("case: alloc failure gk_create")
    fail_at(1)
    try:
        with pytest.raises(gk.GkError) as ei:
            gk.gk_create(0)
    finally:
        fail_at(0)
    assert ei.value.status == gk.GK_ENOMEM
    ctx = gk.gk_create(0)
    try:
        _filter_ok(ctx, data)
    finally:
        gk.gk_destroy(ctx)


def test_load_reference(data):
    ref = data[0]
    n = _each_failure(lambda: gk.gk_create(0), lambda c: gk.gk_load_reference(c, ref),
                      lambda c: _filter_ok(c, data, load=False), "gk_load_reference")
    assert n >= 4


def test_load_reference_2bit(data):
    ref = data[0]
    rng = np.random.default_rng(7)
    packed = pack_2bit(ref, gk.GK_READS_SPLIT, rng)
    runs = unknown_runs(ref)

    def call(c):
        gk.gk_load_reference_2bit(c, packed, len(ref), gk.GK_READS_SPLIT, runs)
    n = _each_failure(lambda: gk.gk_create(0), call,
                      lambda c: _filter_ok(c, data, load=False), "gk_load_reference_2bit")
    assert n >= 4


def _mixed_call(data, fn):
    import torch
    ref, ps, ra, rs = data

    def call(c):
        dr = device.encode_reads(c, ps.reads, ps.read_off, max_len=100)
        dp = device.upload_pairs(ps.pair_read, ps.cand_pos)
        fn(c, device.batch_for(dr, dp, e_uniform=E, max_read_len=100))
        torch.cuda.synchronize()
        a, s = device.results(dp)
        assert_same(a, s, ra, rs, "mixed call after the failure was lifted")
    return call


def _loaded_ctx(data):
    def make():
        c = gk.gk_create(0)
        gk.gk_load_reference(c, data[0])
        return c
    return make


def test_filter_mixed(data):
    _each_failure(_loaded_ctx(data), _mixed_call(data, lambda c, b: gk.gk_filter_mixed(c, b)),
                  lambda c: _filter_ok(c, data, load=False), "gk_filter_mixed")


def test_tune_mixed(data):
    _each_failure(_loaded_ctx(data), _mixed_call(data, lambda c, b: gk.gk_tune_mixed(c, b)),
                  lambda c: _filter_ok(c, data, load=False), "gk_tune_mixed")


def test_verify(data):
    import torch
    ref, ps, ra, rs = data
    want = oracle.levenshtein_batch(ps.reads, ps.read_off, ref, ps.pair_read, ps.cand_pos, E,
                                    n_threads=8)

    def call(c):
        dr = device.encode_reads(c, ps.reads, ps.read_off, max_len=100)
        dp = device.upload_pairs(ps.pair_read, ps.cand_pos)
        dist = torch.empty(ps.n_pairs, dtype=torch.int16, device="cuda")
        gk.gk_verify(c, device.batch_for(dr, dp, e_uniform=E, max_read_len=100), None, dist)
        torch.cuda.synchronize()
        got = dist.cpu().numpy().view(np.uint16)
        assert np.array_equal(got, want), "gk_verify after the failure was lifted"
    _each_failure(_loaded_ctx(data), call, lambda c: _filter_ok(c, data, load=False),
                  "gk_verify")


@pytest.mark.parametrize("threads", [0, 2])
@pytest.mark.parametrize("identity", [False, True], ids=["pair_read", "one-per-read"])
@pytest.mark.parametrize("chunk", [0, 1024], ids=["one-chunk", "three-slots"])
def test_filter_host(data, threads, identity, chunk):
    ref, ps, ra, rs = data
    assert np.array_equal(ps.pair_read, np.arange(ps.n_pairs))

    def call(c):
        gk.gk_set_option(c, gk.GK_OPT_HOST_ENCODE_THREADS, threads)
        gk.gk_set_option(c, gk.GK_OPT_HOST_CHUNK_PAIRS, chunk)
        acc = np.full(ps.n_pairs, 0xEE, np.uint8)
        est = np.full(ps.n_pairs, 0x5A5A, np.uint16)
        gk.gk_filter_host(c, ps.reads, ps.read_off, ps.cand_pos, acc, est, max_read_len=100,
                          pair_read=None if identity else ps.pair_read, e_uniform=E)
        assert_same(acc, est, ra, rs, "gk_filter_host after the failure was lifted")
    _each_failure(_loaded_ctx(data), call, lambda c: _filter_ok(c, data, load=False),
                  f"gk_filter_host threads={threads} identity={identity} chunk={chunk}")


def test_server_start(data):
    def call(c):
        srv = gk.gk_server_start(c, 64 << 20, 8, 128, gk.GK_SERVER_BATCHED)
        gk.gk_server_stop(srv)
    _each_failure(_loaded_ctx(data), call, lambda c: _filter_ok(c, data, load=False),
                  "gk_server_start")

// CPU driver for the serving loop's host logic (gk_server.hip built as host
// C++), against a stand-in HIP runtime: no GPU.  tests/test_server_host.py
// builds it plain and under the address / undefined-behaviour and thread
// sanitizers.
//
// The stand-in runtime gives every stream a worker thread that runs its
// operations in order (copies are memcpy; an event fires when its stream
// reaches it; a captured graph replays its recorded operations), and device
// memory is host memory.  The stand-in kernels write, for every pair, a
// fixed function of the pair's position, its read's length and a hash of
// its read's text (which the stand-in encoder stores in the read's first
// packed word), so a pair filtered against the wrong read, position or
// output slot shows up as a mismatch.
//
// Checks: every request's results equal that function on every pair, with
// requests split over many ticks (pair_read given or not), from several
// submitting threads; the sequential mode; cancellation by gk_server_stop;
// and the error paths (an injected failed load or tick) end every wait.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "gk_internal.h"

extern "C" int gk_detail_server_inject_failure(gk_server *s, uint64_t load_at, uint64_t tick_at);

#include "standin_hip.h"

namespace {

std::atomic<int> g_bad_table{0};      // a tick table inconsistent with its parts

}  // namespace

// ---- stand-in kernels -------------------------------------------------------

namespace {

uint32_t text_hash(const uint8_t *p, uint64_t n)
{
    uint32_t h = 2166136261u;
    for (uint64_t i = 0; i < n; ++i)
        h = (h ^ p[i]) * 16777619u;
    return h;
}

// The stand-in filter result of one pair.
void expected(uint32_t h, uint32_t len, uint32_t pos, uint32_t e, uint8_t *acc, uint16_t *est)
{
    *acc = (uint8_t)((h ^ pos ^ e) & 1u);
    *est = (uint16_t)((h + 3u * pos + 17u * len + e) & 0xFFFEu);
}

void fake_filter(const gkd::FilterArgs &a)
{
    for (uint64_t i = 0; i < a.n_pairs; ++i) {
        const uint32_t r = a.pair_read ? a.pair_read[i] : (uint32_t)i;
        if (r >= a.n_reads) {
            a.accept[i] = GK_INVALID;
            a.est[i] = GK_EST_NONE;
            continue;
        }
        expected(a.reads[r], a.read_len[r], a.cand_pos[i], a.e_uniform, &a.accept[i], &a.est[i]);
    }
}

}  // namespace

namespace gkd {

hipError_t launch_encode_reads(const uint8_t *ascii, const uint64_t *read_off, uint32_t n_reads,
                               uint32_t pitch, uint32_t rows, uint32_t, uint32_t *packed,
                               uint16_t *len_out, uint8_t *has_n_out, hipStream_t s,
                               uint64_t text_base)
{
    s->enqueue([=] {
        for (uint32_t r = 0; r < n_reads; ++r) {
            const uint64_t len = read_off[r + 1] - read_off[r];
            packed[r] = text_hash(ascii + (read_off[r] - text_base), len);
            for (uint32_t w = 1; w < rows; ++w)
                packed[(size_t)w * pitch + r] = 0;
            len_out[r] = (uint16_t)len;
            if (has_n_out)
                has_n_out[r] = 0;
        }
    });
    return hipSuccess;
}

hipError_t launch_filter(const FilterArgs &a, uint32_t, uint32_t, uint32_t, hipStream_t s)
{
    const FilterArgs c = a;
    s->enqueue([c] { fake_filter(c); });
    return hipSuccess;
}

hipError_t launch_mixed_table(const MixedArgs &x, uint32_t, uint32_t, hipStream_t s)
{
    const MixedArgs c = x;
    s->enqueue([c] {
        const BatchTable *t = c.table;
        uint32_t tiles = 0;
        for (uint32_t b = 0; b < t->n_batches; ++b) {
            if (t->prefix[b] != tiles)
                g_bad_table++;
            fake_filter(t->args[b]);
            tiles += (uint32_t)((t->args[b].n_pairs + c.tile - 1) / c.tile);
        }
        if (t->prefix[t->n_batches] != tiles || t->n_batches > MAX_TABLE_BATCHES)
            g_bad_table++;
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    });
    return hipSuccess;
}

hipError_t mixed_blocks_per_cu(uint32_t, uint32_t, uint32_t, uint32_t, int *out)
{
    *out = 4;
    return hipSuccess;
}

}  // namespace gkd

// ---- driver -----------------------------------------------------------------

namespace {

struct TestReq {
    std::vector<uint8_t> text;
    std::vector<uint64_t> off;
    std::vector<uint32_t> pair_read, pos;
    uint32_t e = 0;
    std::vector<uint8_t> acc;
    std::vector<uint16_t> est;
    std::vector<uint8_t> want_acc;
    std::vector<uint16_t> want_est;
};

TestReq make_req(std::mt19937_64 &rng, uint64_t n_pairs, bool identity)
{
    TestReq q;
    const uint32_t n_reads = identity ? (uint32_t)n_pairs
                                      : (uint32_t)std::max<uint64_t>(1, n_pairs / 5 + 1);
    q.off.push_back(0);
    for (uint32_t r = 0; r < n_reads; ++r) {
        const uint32_t len = 60 + (uint32_t)(rng() % 190);
        for (uint32_t j = 0; j < len; ++j)
            q.text.push_back("ACGT"[rng() & 3]);
        q.off.push_back(q.text.size());
    }
    q.e = (uint32_t)(rng() % 20);
    for (uint64_t i = 0; i < n_pairs; ++i) {
        q.pair_read.push_back(identity ? (uint32_t)i : (uint32_t)(rng() % n_reads));
        q.pos.push_back((uint32_t)(rng() % 1000000));
    }
    q.acc.assign(n_pairs, 0xEE);
    q.est.assign(n_pairs, 0x5A5A);
    q.want_acc.resize(n_pairs);
    q.want_est.resize(n_pairs);
    for (uint64_t i = 0; i < n_pairs; ++i) {
        const uint32_t r = q.pair_read[i];
        const uint64_t len = q.off[r + 1] - q.off[r];
        expected(text_hash(q.text.data() + q.off[r], len), (uint32_t)len, q.pos[i], q.e,
                 &q.want_acc[i], &q.want_est[i]);
    }
    return q;
}

gk_request as_request(TestReq &q, bool identity)
{
    gk_request r{};
    r.reads = reinterpret_cast<const char *>(q.text.data());
    r.read_off = q.off.data();
    r.n_reads = (uint32_t)(q.off.size() - 1);
    r.e = q.e;
    r.pair_read = identity ? nullptr : q.pair_read.data();
    r.cand_pos = q.pos.data();
    r.n_pairs = q.pos.size();
    r.accept = q.acc.data();
    r.est = q.est.data();
    r.t_arrival_us = 0;
    return r;
}

int g_failures = 0;

#define CHECK(c, ...)                                                                         \
    do {                                                                                      \
        if (!(c)) {                                                                           \
            std::printf("FAIL %s:%d: ", __FILE__, __LINE__);                                   \
            std::printf(__VA_ARGS__);                                                         \
            std::printf("\n");                                                                \
            g_failures++;                                                                     \
        }                                                                                     \
    } while (0)

// Submit every request from `threads` threads (request k from thread k %
// threads), wait for all, and compare.  Returns the number of ticks.
uint64_t run_batch(gk_ctx *ctx, uint32_t mode, std::vector<TestReq> &reqs,
                   const std::vector<bool> &identity, unsigned threads, uint64_t budget,
                   uint32_t slots, const char *label)
{
    gk_server *srv = nullptr;
    int st = gk_server_start(ctx, budget, slots, 256, mode, &srv);
    CHECK(st == GK_OK, "%s: start %d", label, st);
    if (st != GK_OK)
        return 0;
    std::vector<std::thread> th;
    for (unsigned t = 0; t < threads; ++t)
        th.emplace_back([&, t] {
            std::vector<uint64_t> tickets;
            for (size_t k = t; k < reqs.size(); k += threads) {
                gk_request r = as_request(reqs[k], identity[k]);
                uint64_t ticket = 0;
                const int s = gk_server_submit(srv, &r, &ticket);
                CHECK(s == GK_OK, "%s: submit %zu -> %d", label, k, s);
                tickets.push_back(s == GK_OK ? ticket : 0);
                if ((k / threads) % 3 == 0)
                    std::this_thread::sleep_for(std::chrono::microseconds(50));
            }
            for (uint64_t ticket : tickets) {
                if (!ticket)
                    continue;
                gk_request_stats stats{};
                const int s = gk_server_wait(srv, ticket, 60000000, &stats);
                CHECK(s == GK_OK, "%s: wait -> %d", label, s);
                CHECK(stats.t_done_us >= stats.t_admit_us && stats.t_admit_us >= stats.t_submit_us,
                      "%s: times out of order (submit %lld admit %lld done %lld)", label,
                      (long long)stats.t_submit_us, (long long)stats.t_admit_us,
                      (long long)stats.t_done_us);
            }
        });
    for (auto &t : th)
        t.join();
    uint64_t ticks = 0, max_parts = 0, pairs = 0;
    gk_server_counters(srv, &ticks, &max_parts, &pairs);
    st = gk_server_stop(srv);
    CHECK(st == GK_OK, "%s: stop %d", label, st);
    uint64_t total = 0;
    for (size_t k = 0; k < reqs.size(); ++k) {
        TestReq &q = reqs[k];
        total += q.pos.size();
        size_t bad = 0, first = 0;
        for (size_t i = 0; i < q.pos.size(); ++i)
            if (q.acc[i] != q.want_acc[i] || q.est[i] != q.want_est[i]) {
                if (!bad)
                    first = i;
                bad++;
            }
        CHECK(bad == 0, "%s: request %zu: %zu of %zu pairs wrong, first %zu", label, k, bad,
              q.pos.size(), first);
        std::fill(q.acc.begin(), q.acc.end(), 0xEE);
        std::fill(q.est.begin(), q.est.end(), 0x5A5A);
    }
    CHECK(pairs == total, "%s: pairs_done %llu of %llu", label, (unsigned long long)pairs,
          (unsigned long long)total);
    std::printf("%s: %zu requests, %llu pairs, %llu ticks, at most %llu parts per tick\n", label,
                reqs.size(), (unsigned long long)total, (unsigned long long)ticks,
                (unsigned long long)max_parts);
    return ticks;
}

// An injected failure (load number load_at, or completed tick tick_at):
// every wait returns, with GK_OK or GK_EDEVICE, and OK results are right.
void run_failure(gk_ctx *ctx, std::vector<TestReq> &reqs, uint64_t load_at, uint64_t tick_at)
{
    gk_server *srv = nullptr;
    int st = gk_server_start(ctx, 1ull << 26, 16, 256, GK_SERVER_BATCHED, &srv);
    CHECK(st == GK_OK, "failure: start %d", st);
    if (st != GK_OK)
        return;
    gk_detail_server_inject_failure(srv, load_at, tick_at);
    std::vector<uint64_t> tickets;
    for (auto &q : reqs) {
        gk_request r = as_request(q, false);
        uint64_t t = 0;
        const int s = gk_server_submit(srv, &r, &t);
        CHECK(s == GK_OK || s == GK_EDEVICE, "failure: submit %d", s);
        tickets.push_back(s == GK_OK ? t : 0);
    }
    size_t ok = 0, dev = 0;
    for (size_t k = 0; k < reqs.size(); ++k) {
        if (!tickets[k])
            continue;
        const int s = gk_server_wait(srv, tickets[k], 60000000, nullptr);
        CHECK(s == GK_OK || s == GK_EDEVICE, "failure: wait %d", s);
        if (s == GK_OK) {
            ok++;
            TestReq &q = reqs[k];
            for (size_t i = 0; i < q.pos.size(); ++i)
                if (q.acc[i] != q.want_acc[i] || q.est[i] != q.want_est[i]) {
                    CHECK(false, "failure: OK request %zu has a wrong pair %zu", k, i);
                    break;
                }
        } else {
            dev++;
        }
    }
    st = gk_server_stop(srv);
    CHECK(st == GK_EDEVICE, "failure: stop after a failure %d", st);
    CHECK(dev > 0, "failure: no request saw the failure");
    std::printf("failure load_at=%llu tick_at=%llu: %zu ok, %zu failed\n",
                (unsigned long long)load_at, (unsigned long long)tick_at, ok, dev);
}

}  // namespace

int main()
{
    gk_ctx ctx;
    ctx.device = 0;
    ctx.cu_count = 4;
    static uint2 fake_planes[4];
    ctx.ref_planes = fake_planes;
    ctx.ref_len = 1000000;
    std::mt19937_64 rng(12345);

    std::vector<TestReq> reqs;
    std::vector<bool> identity;
    for (int k = 0; k < 48; ++k) {
        const bool id = k % 3 == 0;
        const uint64_t n = k % 11 == 0 ? 0 : (k % 7 == 0 ? 20000 + rng() % 20000 : rng() % 3000);
        reqs.push_back(make_req(rng, n, id));
        identity.push_back(id);
    }

    // Default parts (no request is split) and tiny parts and ticks (every
    // large request spread over many ticks), with several submitters.
    run_batch(&ctx, GK_SERVER_BATCHED, reqs, identity, 4, 1ull << 28, 64, "batched default");
    ctx.server_part_pairs = 256;
    ctx.server_tick_pairs = 4096;
    const uint64_t ticks =
        run_batch(&ctx, GK_SERVER_BATCHED, reqs, identity, 4, 1ull << 28, 64, "batched split");
    uint64_t total = 0;
    for (auto &q : reqs)
        total += q.pos.size();
    CHECK(ticks >= total / 4096, "split run took only %llu ticks", (unsigned long long)ticks);
    // The loader's copy streams taken in turn: two, and one, with random
    // delays before every stream operation.
    g_jitter_us = 20;
    ctx.server_copy_streams = 2;
    run_batch(&ctx, GK_SERVER_BATCHED, reqs, identity, 4, 1ull << 28, 64,
              "batched split, 2 copy streams, delays");
    ctx.server_copy_streams = 1;
    run_batch(&ctx, GK_SERVER_BATCHED, reqs, identity, 4, 1ull << 28, 64,
              "batched split, 1 copy stream, delays");
    ctx.server_copy_streams = 4;
    g_jitter_us = 0;
    ctx.mixed.tile = 8192;
    ctx.server_part_pairs = 3000;
    ctx.server_tick_pairs = 10000;
    run_batch(&ctx, GK_SERVER_BATCHED, reqs, identity, 3, 1ull << 24, 3,
              "batched split, small budget and 3 slots");
    ctx.mixed.tile = 4096;
    run_batch(&ctx, GK_SERVER_SEQUENTIAL, reqs, identity, 2, 1ull << 28, 8, "sequential");

    // Stop with requests still queued: queued ones are cancelled, admitted
    // ones finish, every wait returns.
    {
        gk_server *srv = nullptr;
        CHECK(gk_server_start(&ctx, 1ull << 28, 2, 256, GK_SERVER_BATCHED, &srv) == GK_OK,
              "stop: start");
        std::vector<uint64_t> tickets;
        for (size_t k = 0; k < reqs.size(); ++k) {
            gk_request r = as_request(reqs[k], identity[k]);
            uint64_t t = 0;
            CHECK(gk_server_submit(srv, &r, &t) == GK_OK, "stop: submit");
            tickets.push_back(t);
        }
        std::thread waiter([&] {
            for (uint64_t t : tickets) {
                const int s = gk_server_wait(srv, t, 60000000, nullptr);
                CHECK(s == GK_OK || s == GK_ECANCELED || s == GK_EINVAL, "stop: wait %d", s);
            }
        });
        std::this_thread::sleep_for(std::chrono::milliseconds(2));
        waiter.join();
        CHECK(gk_server_stop(srv) == GK_OK, "stop: stop");
    }

    ctx.server_part_pairs = 1000;
    ctx.server_tick_pairs = 4096;
    run_failure(&ctx, reqs, 9, 0);
    run_failure(&ctx, reqs, 0, 3);
    run_failure(&ctx, reqs, 0, 40);

    CHECK(g_bad_table.load() == 0, "%d tick tables disagree with their parts",
          g_bad_table.load());
    if (g_failures) {
        std::printf("server check: %d failures\n", g_failures);
        return 1;
    }
    std::printf("server check ok\n");
    return 0;
}

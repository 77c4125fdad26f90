// CPU driver for the served-bench load generator (gk_loadgen.cpp), linked
// against a stand-in server instead of libgk: no GPU.  The stand-in serves
// each request on a worker thread after a short delay, writing outputs that
// are a fixed function of the request's positions.  Checks, under the
// sanitizers tests/test_loadgen.py builds this with:
//   - every submission finishes and its own buffer matches the expected
//     outputs (no mismatches);
//   - a result the server never writes is caught by the sentinel;
//   - one wrong pair is counted as one mismatch;
//   - a request that never finishes is reported unfinished and the run
//     returns at its deadline.
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "gk.h"

extern "C" {
typedef struct gkl_pool_entry {
    const char *reads;
    const uint64_t *read_off;
    uint32_t n_reads;
    uint32_t e;
    const uint32_t *pair_read;
    const uint32_t *cand_pos;
    uint64_t n_pairs;
    const uint8_t *want_accept;
    const uint16_t *want_est;
} gkl_pool_entry;
typedef struct gkl_run_args {
    gk_server *srv;
    const gkl_pool_entry *pool;
    uint32_t n_pool;
    uint32_t n_slots;
    uint64_t slot_pairs;
    uint8_t *ring_accept;
    uint16_t *ring_est;
    uint64_t n_sub;
    const int64_t *arrival_us;
    const uint32_t *which;
    int64_t deadline_us;
    int64_t t_start_us;
} gkl_run_args;
typedef struct gkl_sub_result {
    int32_t status;
    int32_t submit_status;
    int64_t t_arrival_us;
    int64_t t_submit_us;
    int64_t t_admit_us;
    int64_t t_done_us;
    uint64_t n_pairs;
    uint64_t mismatches;
    uint32_t checked;
    uint32_t slot;
} gkl_sub_result;
int gkl_run(gkl_run_args *a, gkl_sub_result *res);
}

static uint8_t out_acc(uint32_t pos, uint32_t e) { return (uint8_t)((pos + e) & 1u); }
static uint16_t out_est(uint32_t pos) { return (uint16_t)(pos & 0x7FFFu); }

// ---- stand-in server --------------------------------------------------------
struct SReq {
    gk_request r;
    bool done = false;
    int64_t t_admit = 0, t_done = 0;
};

struct gk_server {
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> queue;
    std::vector<SReq *> reqs;         // by ticket - 1
    bool stop = false;
    uint64_t drop_ticket = 0;         // never written (sentinel stays)
    uint64_t corrupt_ticket = 0;      // one pair written wrong
    uint64_t hang_ticket = 0;         // never finishes
    std::thread worker;
};

extern "C" int64_t gk_clock_us(void)
{
    return std::chrono::duration_cast<std::chrono::microseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

static void serve(gk_server *s)
{
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        s->cv.wait(lk, [&] { return s->stop || !s->queue.empty(); });
        if (s->stop)
            return;
        const uint64_t t = s->queue.front();
        s->queue.pop_front();
        SReq *q = s->reqs[t - 1];
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(200));
        q->t_admit = gk_clock_us();
        if (t != s->drop_ticket && t != s->hang_ticket) {
            for (uint64_t i = 0; i < q->r.n_pairs; ++i) {
                q->r.accept[i] = out_acc(q->r.cand_pos[i], q->r.e);
                q->r.est[i] = out_est(q->r.cand_pos[i]);
            }
            if (t == s->corrupt_ticket)
                q->r.est[q->r.n_pairs / 2] ^= 1u;
        }
        lk.lock();
        if (t != s->hang_ticket) {
            q->t_done = gk_clock_us();
            q->done = true;
        }
        s->cv.notify_all();
    }
}

extern "C" int gk_server_submit(gk_server *s, const gk_request *r, uint64_t *ticket)
{
    std::lock_guard<std::mutex> lk(s->mu);
    SReq *q = new SReq();
    q->r = *r;
    s->reqs.push_back(q);
    *ticket = s->reqs.size();
    s->queue.push_back(*ticket);
    s->cv.notify_all();
    return GK_OK;
}

extern "C" int gk_server_wait(gk_server *s, uint64_t ticket, int64_t timeout_us,
                              gk_request_stats *st)
{
    std::unique_lock<std::mutex> lk(s->mu);
    SReq *q = s->reqs[ticket - 1];
    // system clock: pthread_cond_timedwait, which the thread sanitizer sees
    if (!s->cv.wait_until(lk, std::chrono::system_clock::now() +
                                  std::chrono::microseconds(timeout_us),
                          [&] { return q->done; }))
        return GK_ETIMEOUT;
    st->status = GK_OK;
    st->n_pairs = q->r.n_pairs;
    st->t_admit_us = q->t_admit;
    st->t_done_us = q->t_done;
    return GK_OK;
}

// ---- driver -------------------------------------------------------------------
static int run_case(const char *name, uint64_t drop, uint64_t corrupt, uint64_t hang,
                    uint64_t want_bad_subs, uint64_t want_unfinished)
{
    const uint32_t n_pool = 5;
    std::vector<std::vector<uint32_t>> pos(n_pool);
    std::vector<std::vector<uint8_t>> wa(n_pool);
    std::vector<std::vector<uint16_t>> we(n_pool);
    std::vector<gkl_pool_entry> pool(n_pool);
    static const char reads[] = "ACGT";
    static const uint64_t off[2] = {0, 4};
    for (uint32_t p = 0; p < n_pool; ++p) {
        const uint64_t n = 100 + 977 * p;
        pos[p].resize(n);
        wa[p].resize(n);
        we[p].resize(n);
        for (uint64_t i = 0; i < n; ++i) {
            pos[p][i] = (uint32_t)(i * 2654435761u + p);
            wa[p][i] = out_acc(pos[p][i], p);
            we[p][i] = out_est(pos[p][i]);
        }
        pool[p] = gkl_pool_entry{reads, off, 1, p, nullptr, pos[p].data(), n, wa[p].data(),
                                 we[p].data()};
    }
    const uint32_t n_slots = 4;
    const uint64_t slot_pairs = 100 + 977 * (n_pool - 1);
    std::vector<uint8_t> ring_a(n_slots * slot_pairs);
    std::vector<uint16_t> ring_e(n_slots * slot_pairs);
    const uint64_t n_sub = 60;
    std::vector<int64_t> arr(n_sub);
    std::vector<uint32_t> which(n_sub);
    for (uint64_t k = 0; k < n_sub; ++k) {
        arr[k] = (int64_t)(k * 150);
        which[k] = (uint32_t)((k * 7) % n_pool);
    }
    gk_server srv;
    srv.drop_ticket = drop;
    srv.corrupt_ticket = corrupt;
    srv.hang_ticket = hang;
    srv.worker = std::thread(serve, &srv);
    gkl_run_args a{};
    a.srv = &srv;
    a.pool = pool.data();
    a.n_pool = n_pool;
    a.n_slots = n_slots;
    a.slot_pairs = slot_pairs;
    a.ring_accept = ring_a.data();
    a.ring_est = ring_e.data();
    a.n_sub = n_sub;
    a.arrival_us = arr.data();
    a.which = which.data();
    a.deadline_us = 2000000;
    std::vector<gkl_sub_result> res(n_sub);
    const int st = gkl_run(&a, res.data());
    // Nothing may touch the ring after the server stops.
    {
        std::lock_guard<std::mutex> lk(srv.mu);
        srv.stop = true;
        srv.cv.notify_all();
    }
    srv.worker.join();
    for (SReq *q : srv.reqs)
        delete q;
    uint64_t bad = 0, unfinished = 0, total_bad_pairs = 0;
    for (uint64_t k = 0; k < n_sub; ++k) {
        if (res[k].status != GK_OK)
            ++unfinished;
        else if (res[k].mismatches)
            ++bad;
        total_bad_pairs += res[k].mismatches;
    }
    const bool ok = st == GK_OK && bad == want_bad_subs && unfinished == want_unfinished &&
                    (corrupt == 0 || total_bad_pairs >= 1);
    std::printf("%s: status %d, mismatched submissions %llu (want %llu), unfinished %llu "
                "(want %llu) -> %s\n",
                name, st, (unsigned long long)bad, (unsigned long long)want_bad_subs,
                (unsigned long long)unfinished, (unsigned long long)want_unfinished,
                ok ? "ok" : "FAIL");
    return ok ? 0 : 1;
}

int main()
{
    int fails = 0;
    fails += run_case("clean", 0, 0, 0, 0, 0);
    fails += run_case("dropped result", 7, 0, 0, 1, 0);
    fails += run_case("one wrong pair", 0, 11, 0, 1, 0);
    // The 40th submission never finishes: the in-order waiter stops there at
    // the deadline, so it and every later submission are unfinished.
    fails += run_case("never finishes", 0, 0, 40, 0, 21);
    if (fails == 0)
        std::printf("loadgen check ok\n");
    return fails ? 1 : 0;
}

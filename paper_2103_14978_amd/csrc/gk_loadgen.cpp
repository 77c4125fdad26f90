// Open-loop load generator for the serving loop (measurement support, not
// part of the filter): submits pool requests to a gk_server at scheduled
// arrival times from a native thread (no interpreter lock between the
// schedule and gk_server_submit), waits for them in submission order on the
// calling thread, and checks each submission's own outputs against the
// expected outputs of its pool request.  Built into libgk_loadgen.so.
//
// Outputs land in a ring of caller-owned host buffers, one per submission in
// flight.  A buffer is filled with a sentinel (accept 0xFF, est 0xFFFF)
// before it is handed to a submission, so a result that never arrived counts
// as a mismatch.  A submission that finds no free buffer waits for one; its
// latency still runs from its scheduled arrival.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "gk.h"

extern "C" {

typedef struct gkl_pool_entry {
    const char *reads;            // HOST ASCII, as gk_request.reads
    const uint64_t *read_off;     // HOST n_reads + 1 offsets
    uint32_t n_reads;
    uint32_t e;
    const uint32_t *pair_read;    // HOST n_pairs or NULL
    const uint32_t *cand_pos;     // HOST n_pairs
    uint64_t n_pairs;
    const uint8_t *want_accept;   // HOST n_pairs expected codes, or NULL (unchecked)
    const uint16_t *want_est;     // HOST n_pairs expected estimates (with want_accept)
} gkl_pool_entry;

typedef struct gkl_run_args {
    gk_server *srv;
    const gkl_pool_entry *pool;
    uint32_t n_pool;
    uint32_t n_slots;             // output buffers in the ring (>= 1)
    uint64_t slot_pairs;          // pairs per buffer (>= every pool request)
    uint8_t *ring_accept;         // HOST n_slots * slot_pairs
    uint16_t *ring_est;           // HOST n_slots * slot_pairs
    uint64_t n_sub;
    const int64_t *arrival_us;    // n_sub scheduled arrivals, microseconds after the
                                  // start, non-decreasing
    const uint32_t *which;        // n_sub pool indices
    int64_t deadline_us;          // microseconds after the start: no wait extends past it
    int64_t t_start_us;           // out: the start on gk_clock_us()'s clock, set 200 ms
                                  // after the ring is filled with the sentinel
} gkl_run_args;

// Per submission.  status: the wait's GK_* status, or GKL_UNFINISHED (still
// running at the deadline), or GKL_NOT_SUBMITTED (no buffer before the
// deadline, or a refused submit: then submit_status holds its code).
#define GKL_UNFINISHED    1
#define GKL_NOT_SUBMITTED 2
typedef struct gkl_sub_result {
    int32_t status;
    int32_t submit_status;
    int64_t t_arrival_us;         // scheduled arrival
    int64_t t_submit_us;          // gk_server_submit called
    int64_t t_admit_us;           // from gk_request_stats
    int64_t t_done_us;            // results in the host buffer
    uint64_t n_pairs;
    uint64_t mismatches;          // pairs differing from the expected outputs
    uint32_t checked;             // 1 if the pool request had expected outputs
    uint32_t slot;
} gkl_sub_result;

}  // extern "C"

namespace {

struct Inflight {
    uint64_t k;        // submission index
    uint64_t ticket;
    uint32_t slot;
};

// Timed wait on the system clock (pthread_cond_timedwait), which the thread
// sanitizer's interceptors see; waits are bounded by the run's deadline.
void wait_for_us(std::condition_variable &cv, std::unique_lock<std::mutex> &lk, int64_t us)
{
    cv.wait_until(lk, std::chrono::system_clock::now() + std::chrono::microseconds(us));
}

void fill_sentinel(const gkl_run_args *a, uint32_t slot, uint64_t n)
{
    std::memset(a->ring_accept + (uint64_t)slot * a->slot_pairs, 0xFF, n);
    std::memset(a->ring_est + (uint64_t)slot * a->slot_pairs, 0xFF, 2 * n);
}

}  // namespace

extern "C" {

// Runs the schedule; returns 0, or GK_EINVAL for bad arguments.  The server
// may still hold buffers of unfinished submissions when this returns: stop
// the server (gk_server_stop) before the ring is freed.
int gkl_run(gkl_run_args *a, gkl_sub_result *res)
{
    if (!a || !res || !a->srv || !a->pool || a->n_pool == 0 || a->n_slots == 0 ||
        !a->ring_accept || !a->ring_est || (a->n_sub && (!a->arrival_us || !a->which)))
        return GK_EINVAL;
    for (uint32_t p = 0; p < a->n_pool; ++p)
        if (a->pool[p].n_pairs > a->slot_pairs)
            return GK_EINVAL;
    for (uint64_t k = 0; k < a->n_sub; ++k)
        if (a->which[k] >= a->n_pool)
            return GK_EINVAL;
    for (uint32_t s = 0; s < a->n_slots; ++s)
        fill_sentinel(a, s, a->slot_pairs);
    const int64_t t0 = gk_clock_us() + 200000;
    a->t_start_us = t0;
    const int64_t deadline = t0 + a->deadline_us;
    std::memset(res, 0, a->n_sub * sizeof(gkl_sub_result));
    for (uint64_t k = 0; k < a->n_sub; ++k) {
        res[k].status = GKL_NOT_SUBMITTED;
        res[k].t_arrival_us = t0 + a->arrival_us[k];
        res[k].n_pairs = a->pool[a->which[k]].n_pairs;
    }

    std::mutex mu;
    std::condition_variable cv;
    std::vector<uint32_t> free_slots;
    for (uint32_t s = a->n_slots; s-- > 0;)
        free_slots.push_back(s);
    std::deque<Inflight> q;
    bool sub_done = false;
    std::atomic<bool> stop{false};

    std::thread submitter([&] {
        for (uint64_t k = 0; k < a->n_sub; ++k) {
            const int64_t arrival = res[k].t_arrival_us;
            if (arrival >= deadline)
                break;
            // Sleep to within 200 us of the arrival (a millisecond at a
            // time, watching for the stop), then spin.
            while (!stop.load()) {
                const int64_t d = arrival - gk_clock_us();
                if (d <= 0)
                    break;
                if (d > 300)
                    std::this_thread::sleep_for(
                        std::chrono::microseconds(d - 200 < 1000 ? d - 200 : 1000));
            }
            if (stop.load())
                break;
            uint32_t slot = 0;
            {
                std::unique_lock<std::mutex> lk(mu);
                while (free_slots.empty() && !stop.load()) {
                    const int64_t left = deadline - gk_clock_us();
                    if (left <= 0)
                        break;
                    wait_for_us(cv, lk, left);
                }
                if (stop.load() || free_slots.empty())
                    break;
                slot = free_slots.back();
                free_slots.pop_back();
            }
            const gkl_pool_entry &p = a->pool[a->which[k]];
            gk_request r{};
            r.reads = p.reads;
            r.read_off = p.read_off;
            r.n_reads = p.n_reads;
            r.e = p.e;
            r.pair_read = p.pair_read;
            r.cand_pos = p.cand_pos;
            r.n_pairs = p.n_pairs;
            r.accept = a->ring_accept + (uint64_t)slot * a->slot_pairs;
            r.est = a->ring_est + (uint64_t)slot * a->slot_pairs;
            r.t_arrival_us = arrival;
            uint64_t ticket = 0;
            res[k].t_submit_us = gk_clock_us();
            res[k].slot = slot;
            const int st = gk_server_submit(a->srv, &r, &ticket);
            std::lock_guard<std::mutex> lk(mu);
            if (st != GK_OK) {
                res[k].submit_status = st;
                free_slots.push_back(slot);
                break;
            }
            res[k].status = GKL_UNFINISHED;
            q.push_back(Inflight{k, ticket, slot});
            cv.notify_all();
        }
        std::lock_guard<std::mutex> lk(mu);
        sub_done = true;
        cv.notify_all();
    });

    // Waiter: tickets in submission order.
    while (true) {
        Inflight f{};
        {
            std::unique_lock<std::mutex> lk(mu);
            while (q.empty() && !sub_done) {
                const int64_t left = deadline - gk_clock_us();
                if (left <= 0)
                    break;
                wait_for_us(cv, lk, left);
            }
            if (q.empty())
                break;
            f = q.front();
        }
        const int64_t left = deadline - gk_clock_us();
        if (left <= 0)
            break;
        gk_request_stats st{};
        const int ws = gk_server_wait(a->srv, f.ticket, left, &st);
        if (ws == GK_ETIMEOUT)
            break;
        gkl_sub_result &r = res[f.k];
        r.status = ws;
        r.t_admit_us = st.t_admit_us;
        r.t_done_us = st.t_done_us;
        const gkl_pool_entry &p = a->pool[a->which[f.k]];
        const uint8_t *acc = a->ring_accept + (uint64_t)f.slot * a->slot_pairs;
        const uint16_t *est = a->ring_est + (uint64_t)f.slot * a->slot_pairs;
        if (p.want_accept && p.want_est) {
            r.checked = 1;
            if (std::memcmp(acc, p.want_accept, p.n_pairs) != 0 ||
                std::memcmp(est, p.want_est, 2 * p.n_pairs) != 0) {
                uint64_t bad = 0;
                for (uint64_t i = 0; i < p.n_pairs; ++i)
                    bad += (acc[i] != p.want_accept[i]) | (est[i] != p.want_est[i]);
                r.mismatches = bad;
            }
        }
        fill_sentinel(a, f.slot, p.n_pairs);
        std::lock_guard<std::mutex> lk(mu);
        q.pop_front();
        free_slots.push_back(f.slot);
        cv.notify_all();
    }
    {
        std::lock_guard<std::mutex> lk(mu);
        stop.store(true);
        cv.notify_all();
    }
    submitter.join();
    return GK_OK;
}

}  // extern "C"

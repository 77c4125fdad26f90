// Serving loop for the GateKeeper-GPU filter: admission by device memory and
// slots, request state on the GPU, continuous batching of every loaded
// request into the persistent mixed-batch kernel.
//
// Threads (batched mode):
//   loader     admits pending requests in arrival order when a slot is free
//              and the device arena has room, copies the request in on the
//              copy stream and encodes its reads there (gk_encode_reads'
//              kernel), then marks it ready;
//   scheduler  every tick takes parts of the ready requests in turn (at most
//              part_pairs pairs of one request, at most tick_pairs pairs in
//              all; a request with pairs left goes to the back of the
//              queue), fills a batch table in pinned memory and replays a
//              captured graph on the compute stream (table copy -> reset ->
//              persistent kernel -> residual pass); at most two ticks are in
//              flight, the two table buffers alternate;
//   completer  waits for ticks in order, copies each part's results back,
//              and once a request's last part is back frees its arena range
//              and slot and wakes its waiter.
// So copies of new requests overlap the kernel of the current tick, a
// request arriving while others run joins the next tick, and a large request
// is spread over several ticks instead of holding one: a small request
// behind it waits for one tick, not for the large one's whole run.
//
// Sequential mode (the per-request baseline): the loader alone takes one
// request at a time through copy in, encode, one plain gk_filter launch and
// copy out on a single stream.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gk_internal.h"
#include "gk_trace.h"

namespace {

int64_t now_us()
{
    return std::chrono::duration_cast<std::chrono::microseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

constexpr uint64_t ALIGN = 256;
uint64_t align_up(uint64_t v) { return (v + ALIGN - 1) & ~(ALIGN - 1); }

// First-fit allocator over one device region; free ranges are coalesced.
class Arena {
  public:
    void init(uint64_t size)
    {
        free_.clear();
        free_[0] = size;
        size_ = size;
    }
    bool alloc(uint64_t n, uint64_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const uint64_t rest = it->second - n, at = it->first + n;
                free_.erase(it);
                if (rest)
                    free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t n)
    {
        auto it = free_.emplace(off, n).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t size() const { return size_; }

  private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t size_ = 0;
};

struct Req {
    uint64_t ticket = 0;
    gk_request r{};
    uint32_t max_len = 0, rows = 0, pitch = 0;
    uint64_t ascii_bytes = 0, footprint = 0, arena_off = 0;
    uint8_t *d_ascii = nullptr;
    uint64_t *d_off = nullptr;
    uint32_t *d_packed = nullptr;
    uint16_t *d_len = nullptr;
    uint8_t *d_hasn = nullptr;
    uint32_t *d_pr = nullptr, *d_pos = nullptr;
    uint8_t *d_acc = nullptr;
    uint16_t *d_est = nullptr;
    hipEvent_t ready = nullptr;
    int64_t t_submit = 0, t_admit = 0, t_done = 0;
    int status = GK_OK;
    bool done = false, admitted = false;
    // batched mode: pairs [0, next_pair) are in ticks; live_parts of them
    // are not back yet; failed: a part or the server failed
    uint64_t next_pair = 0;
    uint32_t live_parts = 0;
    bool failed = false;
};

// Pairs [first, first + n) of one request, filtered in one tick.
struct Part {
    Req *q = nullptr;
    uint64_t first = 0, n = 0;
};

struct Tick {
    int buf = 0;
    std::vector<Part> parts;
    int64_t t_launch = 0;
    uint64_t pairs = 0;
};

constexpr size_t TICK_LOG_CAP = 1u << 20;   // tick records kept per server

}  // namespace

struct gk_server {
    gk_ctx *ctx = nullptr;
    uint32_t mode = GK_SERVER_BATCHED;
    uint32_t max_slots = 0, max_read_len = 0, wmax = 0;
    uint64_t budget = 0;
    Arena arena;
    uint8_t *d_arena = nullptr;
    // Copy streams: the loader takes them in turn in batched mode, so one
    // request's transfers and encoding overlap the next ones'; sequential
    // mode uses the first alone.
    static constexpr uint32_t MAX_COPY_STREAMS = 8;
    hipStream_t s_copy[MAX_COPY_STREAMS] = {};
    uint32_t n_copy = 1;
    hipStream_t s_compute = nullptr, s_d2h = nullptr;
    uint64_t admitted = 0;                 // requests admitted so far
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req *> pending, ready;
    std::deque<Tick> inflight;
    std::unordered_map<uint64_t, Req *> reqs;
    uint32_t slots_used = 0;
    uint64_t next_ticket = 1;
    bool stopping = false;
    std::string err;
    std::thread loader, scheduler, completer;
    // tick resources, double-buffered
    gkd::BatchTable *h_table[2] = {nullptr, nullptr};
    gkd::BatchTable *d_table[2] = {nullptr, nullptr};
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    hipEvent_t tick_done[2] = {nullptr, nullptr};
    bool buf_busy[2] = {false, false};
    uint32_t *d_counters = nullptr;
    uint32_t *d_resid = nullptr;
    gkd::MixedArgs margs{};
    uint64_t part_pairs = 0, tick_pairs = 0;   // batched mode: part and tick bounds
    uint64_t ticks = 0, tick_req_max = 0, pairs_done = 0;
    std::vector<gk_tick_record> tick_log;  // first TICK_LOG_CAP ticks, in order
    int tick_buf = 0;
    bool completing = false;               // the completer holds inflight.front()
    // Failure injection for tests of the error paths, with no GPU fault: the
    // loader's k-th load, or the completer's k-th tick, reports an error as a
    // failed HIP call would (0 = never).
    uint64_t fail_load_at = 0, fail_tick_at = 0, loads = 0, ticks_taken = 0;
};

namespace {

// Device footprint of a request, laid out in this order inside its arena
// range: ASCII, offsets, packed reads, lengths, unknown flags, pair reads,
// positions, accept codes, estimates.
void plan(Req *q)
{
    const gk_request &r = q->r;
    q->ascii_bytes = r.read_off[r.n_reads];
    uint32_t mx = 1;
    for (uint32_t i = 0; i < r.n_reads; ++i) {
        const uint64_t len = r.read_off[i + 1] - r.read_off[i];
        if (len > mx)
            mx = (uint32_t)(len < 0xFFFFu ? len : 0xFFFFu);
    }
    q->max_len = mx;
    q->rows = (mx + 15) / 16;
    q->pitch = (r.n_reads + 63) / 64 * 64;
    q->footprint = align_up(q->ascii_bytes ? q->ascii_bytes : 4) +
                   align_up(8ull * (r.n_reads + 1)) + align_up(4ull * q->rows * q->pitch) +
                   align_up(2ull * r.n_reads) + align_up(r.n_reads) +
                   (r.pair_read ? align_up(4 * r.n_pairs) : 0) + align_up(4 * r.n_pairs) +
                   align_up(r.n_pairs) + align_up(2 * r.n_pairs);
}

void place(gk_server *s, Req *q)
{
    uint8_t *p = s->d_arena + q->arena_off;
    const gk_request &r = q->r;
    q->d_ascii = p;
    p += align_up(q->ascii_bytes ? q->ascii_bytes : 4);
    q->d_off = (uint64_t *)p;
    p += align_up(8ull * (r.n_reads + 1));
    q->d_packed = (uint32_t *)p;
    p += align_up(4ull * q->rows * q->pitch);
    q->d_len = (uint16_t *)p;
    p += align_up(2ull * r.n_reads);
    q->d_hasn = p;
    p += align_up(r.n_reads);
    q->d_pr = nullptr;
    if (r.pair_read) {
        q->d_pr = (uint32_t *)p;
        p += align_up(4 * r.n_pairs);
    }
    q->d_pos = (uint32_t *)p;
    p += align_up(4 * r.n_pairs);
    q->d_acc = p;
    p += align_up(r.n_pairs);
    q->d_est = (uint16_t *)p;
}

// Arguments of pairs [first, first + n) of a request.  With no pair_read
// (pair i uses read i) the read arrays are offset too: the transposed rows
// have stride pitch, so reads + first holds read first + i at column i.
gkd::FilterArgs args_for(const gk_server *s, const Req *q, uint64_t first, uint64_t n)
{
    const gk_ctx *c = s->ctx;
    gkd::FilterArgs a{};
    a.ref_planes = c->ref_planes;
    a.ref_planes_b = c->ref_planes_b;
    a.ref_unk = c->ref_unk;
    a.ref_unk_lines = c->ref_unk_lines;
    a.ref_len = c->ref_len;
    a.ref_has_unknown = c->ref_unknown > 0;
    a.n_reads = q->r.n_reads;
    a.pitch = q->pitch;
    a.e_uniform = q->r.e;
    a.max_read_len = s->max_read_len;
    a.rows = q->rows;
    a.reads = q->d_packed;
    a.read_len = q->d_len;
    a.read_has_n = q->d_hasn;
    a.pair_read = q->d_pr ? q->d_pr + first : nullptr;
    if (!q->d_pr && first > 0) {
        a.n_reads = first < q->r.n_reads ? (uint32_t)(q->r.n_reads - first) : 0u;
        a.reads = q->d_packed + first;
        a.read_len = q->d_len + first;
        a.read_has_n = q->d_hasn + first;
    }
    a.cand_pos = q->d_pos + first;
    a.e_pair = nullptr;
    a.n_pairs = n;
    a.accept = q->d_acc + first;
    a.est = q->d_est + first;
    a.accept_bits = nullptr;
    a.stream_reads = 0;
    return a;
}

// Copy a request in and encode its reads on `st` (caller thread blocks only
// for the pageable host copies).
hipError_t load_request(gk_server *s, Req *q, hipStream_t st)
{
    const gk_request &r = q->r;
    hipError_t e = hipSuccess;
    if (q->ascii_bytes)
        e = hipMemcpyAsync(q->d_ascii, r.reads, q->ascii_bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(q->d_off, r.read_off, 8ull * (r.n_reads + 1), hipMemcpyHostToDevice,
                           st);
    if (e == hipSuccess && r.pair_read)
        e = hipMemcpyAsync(q->d_pr, r.pair_read, 4 * r.n_pairs, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(q->d_pos, r.cand_pos, 4 * r.n_pairs, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = gkd::launch_encode_reads(q->d_ascii, q->d_off, r.n_reads, q->pitch, q->rows,
                                     GK_READS_SPLIT, q->d_packed, q->d_len, q->d_hasn, st);
    return e;
}

// Results of pairs [first, first + n) to the request's host buffers.
hipError_t copy_out(Req *q, uint64_t first, uint64_t n, hipStream_t st)
{
    if (n == 0)
        return hipSuccess;
    hipError_t e =
        hipMemcpyAsync(q->r.accept + first, q->d_acc + first, n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(q->r.est + first, q->d_est + first, 2 * n, hipMemcpyDeviceToHost, st);
    return e;
}

void finish(gk_server *s, Req *q, int status)
{
    // caller holds s->mu
    if (q->done)
        return;
    q->status = status;
    q->t_done = now_us();
    q->done = true;
    if (q->admitted) {
        s->arena.release(q->arena_off, q->footprint);
        s->slots_used--;
        q->admitted = false;
    }
    s->pairs_done += q->r.n_pairs;
}

// Batched mode, caller holds s->mu: a request ends once no part of it is
// out (so no copy can still touch its host buffers) and either all its pairs
// are back or it failed.
void maybe_finish(gk_server *s, Req *q)
{
    if (!q->done && q->live_parts == 0 && (q->failed || q->next_pair >= q->r.n_pairs))
        finish(s, q, q->failed ? GK_EDEVICE : GK_OK);
}

// A part is back (ok) or abandoned after a failure (!ok); caller holds s->mu.
void retire(gk_server *s, const Part &p, bool ok)
{
    p.q->live_parts--;
    if (!ok)
        p.q->failed = true;
    maybe_finish(s, p.q);
}

void fail_all(gk_server *s, const std::string &msg)
{
    // Caller holds s->mu: a device error ends the server's work.  Requests
    // are finished (so their waits return GK_EDEVICE) only once no copy can
    // still touch their host buffers: the copy streams are drained first,
    // and the tick the completer is copying out stays with the completer.
    // The loader and the scheduler finish the requests they hold themselves.
    s->err = msg;
    for (hipStream_t st : s->s_copy)
        if (st)
            (void)hipStreamSynchronize(st);
    // Requests with a part in the tick being completed end when the
    // completer hands that part back.
    for (auto *q : s->pending)
        finish(s, q, GK_EDEVICE);
    for (auto *q : s->ready) {
        q->failed = true;
        maybe_finish(s, q);
    }
    const size_t keep = s->completing && !s->inflight.empty() ? 1 : 0;
    for (size_t i = keep; i < s->inflight.size(); ++i)
        for (const Part &p : s->inflight[i].parts)
            retire(s, p, false);
    s->pending.clear();
    s->ready.clear();
    s->inflight.erase(s->inflight.begin() + keep, s->inflight.end());
    s->stopping = true;
    s->cv.notify_all();
}

void loader_main(gk_server *s)
{
    DeviceScope dev(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        s->cv.wait(lk, [&] { return s->stopping || !s->pending.empty(); });
        if (s->stopping)
            break;
        Req *q = s->pending.front();
        uint64_t off = 0;
        bool got = false;
        // Admission in arrival order: wait for a slot and arena room.  The
        // head may be cancelled meanwhile (gk_server_stop): then start over.
        s->cv.wait(lk, [&] {
            if (s->stopping || s->pending.empty() || s->pending.front() != q)
                return true;
            if (s->slots_used < s->max_slots && s->arena.alloc(q->footprint, &off))
                got = true;
            return got;
        });
        if (s->stopping) {
            if (got)
                s->arena.release(off, q->footprint);
            break;
        }
        if (!got)
            continue;
        s->pending.pop_front();
        s->slots_used++;
        q->admitted = true;
        q->arena_off = off;
        q->t_admit = now_us();
        place(s, q);
        const bool inject = s->fail_load_at != 0 && ++s->loads == s->fail_load_at;
        lk.unlock();

        // Batched mode takes the copy streams in turn.
        const hipStream_t st =
            s->s_copy[s->mode == GK_SERVER_BATCHED ? s->admitted++ % s->n_copy : 0];
        gkd::trace_push("gk_server load");
        hipError_t e = load_request(s, q, st);
        if (e == hipSuccess && inject)
            e = hipErrorInvalidValue;
        if (s->mode == GK_SERVER_SEQUENTIAL) {
            // One request at a time on one stream: copy in, encode, filter, copy out.
            if (e == hipSuccess) {
                const gkd::FilterArgs a = args_for(s, q, 0, q->r.n_pairs);
                e = gkd::launch_filter(a, s->wmax, GK_READS_SPLIT, 0, st);
            }
            if (e == hipSuccess)
                e = copy_out(q, 0, q->r.n_pairs, st);
            const hipError_t es = hipStreamSynchronize(st);   // always drained
            if (e == hipSuccess)
                e = es;
            gkd::trace_pop();
            lk.lock();
            if (e != hipSuccess) {
                finish(s, q, GK_EDEVICE);
                fail_all(s, std::string("server: ") + hipGetErrorName(e));
                break;
            }
            finish(s, q, GK_OK);
            s->cv.notify_all();
            continue;
        }
        if (e == hipSuccess)
            e = hipEventRecord(q->ready, st);
        gkd::trace_pop();
        lk.lock();
        if (e != hipSuccess || s->stopping) {
            // A failure here, or in another thread while this request was
            // loading: its copies are drained before its wait can return.
            lk.unlock();
            (void)hipStreamSynchronize(st);
            lk.lock();
            finish(s, q, GK_EDEVICE);
            if (e != hipSuccess)
                fail_all(s, std::string("server load: ") + hipGetErrorName(e));
            else
                s->cv.notify_all();
            break;
        }
        s->ready.push_back(q);
        s->cv.notify_all();
    }
}

void scheduler_main(gk_server *s)
{
    DeviceScope dev(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        s->cv.wait(lk, [&] {
            return s->stopping || (!s->ready.empty() && !s->buf_busy[s->tick_buf]);
        });
        if (s->stopping)
            break;
        Tick t;
        t.buf = s->tick_buf;
        // Parts in turn: the front request gives at most part_pairs of its
        // pairs (fewer when the tick's budget runs out) and, with pairs
        // left, goes to the back.  At most 256 parts and tick_pairs pairs
        // (tick_pairs <= 2^26: launch-wide pair ids stay below 2^31).  A
        // request with no pairs takes one empty part.
        uint64_t budget = s->tick_pairs;
        while (!s->ready.empty() && t.parts.size() < gkd::MAX_TABLE_BATCHES && budget > 0) {
            Req *q = s->ready.front();
            s->ready.pop_front();
            const uint64_t left = q->r.n_pairs - q->next_pair;
            const uint64_t take = std::min(left, std::min(s->part_pairs, budget));
            t.parts.push_back(Part{q, q->next_pair, take});
            q->next_pair += take;
            q->live_parts++;
            budget -= take;
            t.pairs += take;
            if (q->next_pair < q->r.n_pairs)
                s->ready.push_back(q);
        }
        s->buf_busy[t.buf] = true;
        s->tick_buf ^= 1;
        lk.unlock();

        gkd::trace_push("gk_server tick");
        gkd::BatchTable *h = s->h_table[t.buf];
        h->n_batches = (uint32_t)t.parts.size();
        uint32_t tiles = 0;
        for (size_t b = 0; b < t.parts.size(); ++b) {
            const Part &p = t.parts[b];
            h->prefix[b] = tiles;
            h->args[b] = args_for(s, p.q, p.first, p.n);
            tiles += (uint32_t)((p.n + s->margs.tile - 1) / s->margs.tile);
        }
        h->prefix[t.parts.size()] = tiles;
        hipError_t e = hipSuccess;
        for (const Part &p : t.parts)
            if (e == hipSuccess && p.first == 0)   // a request's loads, once
                e = hipStreamWaitEvent(s->s_compute, p.q->ready, 0);
        t.t_launch = now_us();
        if (e == hipSuccess)
            e = hipGraphLaunch(s->graph[t.buf], s->s_compute);
        if (e == hipSuccess)
            e = hipEventRecord(s->tick_done[t.buf], s->s_compute);
        gkd::trace_pop();
        lk.lock();
        if (e != hipSuccess || s->stopping) {
            // A failure here, or in another thread meanwhile (the completer
            // may have gone): this tick's requests end here, after what was
            // launched for them.
            lk.unlock();
            (void)hipStreamSynchronize(s->s_compute);
            lk.lock();
            for (const Part &p : t.parts)
                retire(s, p, false);
            s->buf_busy[t.buf] = false;
            if (e != hipSuccess)
                fail_all(s, std::string("server tick: ") + hipGetErrorName(e));
            else
                s->cv.notify_all();
            break;
        }
        s->ticks++;
        if (t.parts.size() > s->tick_req_max)
            s->tick_req_max = t.parts.size();
        s->inflight.push_back(std::move(t));
        s->cv.notify_all();
    }
}

void completer_main(gk_server *s)
{
    DeviceScope dev(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        s->cv.wait(lk, [&] { return s->stopping || !s->inflight.empty(); });
        if (s->inflight.empty() && s->stopping)
            break;
        Tick t = s->inflight.front();
        s->completing = true;
        const bool inject = s->fail_tick_at != 0 && ++s->ticks_taken == s->fail_tick_at;
        lk.unlock();
        gkd::trace_push("gk_server complete");
        hipError_t e = hipEventSynchronize(s->tick_done[t.buf]);
        const int64_t t_kernel_done = now_us();
        const bool released = e == hipSuccess;
        if (released) {
            // The tick's kernels are done with its table: the scheduler may
            // launch the next tick into this buffer while the results are
            // copied out (so the buffer must not be released again below).
            lk.lock();
            s->buf_busy[t.buf] = false;
            s->cv.notify_all();
            lk.unlock();
        }
        for (const Part &p : t.parts)
            if (e == hipSuccess)
                e = copy_out(p.q, p.first, p.n, s->s_d2h);
        const hipError_t es = hipStreamSynchronize(s->s_d2h);     // always drained
        if (e == hipSuccess)
            e = es;
        if (e == hipSuccess && inject)
            e = hipErrorInvalidValue;
        const int64_t t_copied = now_us();
        gkd::trace_pop();
        lk.lock();
        if (e == hipSuccess && s->tick_log.size() < TICK_LOG_CAP)
            s->tick_log.push_back(gk_tick_record{t.t_launch, t_kernel_done, t_copied,
                                                 (uint32_t)t.parts.size(), 0u, t.pairs});
        s->completing = false;
        s->inflight.pop_front();     // fail_all leaves the tick being completed
        for (const Part &p : t.parts)
            retire(s, p, e == hipSuccess);
        if (!released)
            s->buf_busy[t.buf] = false;
        if (e != hipSuccess) {
            fail_all(s, std::string("server copy out: ") + hipGetErrorName(e));
            break;
        }
        s->cv.notify_all();
    }
}

void destroy_server(gk_server *s)
{
    DeviceScope dev(s->ctx->device);
    // After a failure, ticks launched before it may still run: nothing the
    // server's streams use is freed before they are drained.
    for (hipStream_t st : s->s_copy)
        if (st)
            (void)hipStreamSynchronize(st);
    for (hipStream_t st : {s->s_compute, s->s_d2h})
        if (st)
            (void)hipStreamSynchronize(st);
    for (int k = 0; k < 2; ++k) {
        if (s->graph[k])
            (void)hipGraphExecDestroy(s->graph[k]);
        if (s->tick_done[k])
            (void)hipEventDestroy(s->tick_done[k]);
        if (s->h_table[k])
            (void)hipHostFree(s->h_table[k]);
        if (s->d_table[k])
            (void)hipFree(s->d_table[k]);
    }
    for (auto &kv : s->reqs) {
        if (kv.second->ready)
            (void)hipEventDestroy(kv.second->ready);
        delete kv.second;
    }
    if (s->d_arena)
        (void)hipFree(s->d_arena);
    if (s->d_counters)
        (void)hipFree(s->d_counters);
    if (s->d_resid)
        (void)hipFree(s->d_resid);
    for (hipStream_t st : s->s_copy)
        if (st)
            (void)hipStreamDestroy(st);
    for (hipStream_t st : {s->s_compute, s->s_d2h})
        if (st)
            (void)hipStreamDestroy(st);
    delete s;
}

}  // namespace

extern "C" {

int gk_server_start(gk_ctx *ctx, uint64_t device_budget_bytes, uint32_t max_slots,
                    uint32_t max_read_len, uint32_t mode, gk_server **out)
{
    if (!ctx || !out)
        return GK_EINVAL;
    *out = nullptr;
    if (!ctx->ref_planes)
        return gk_detail_fail(ctx, GK_ENOREF, "gk_server_start: no reference loaded");
    if (max_slots < 1 || max_slots > gkd::MAX_TABLE_BATCHES)
        return gk_detail_fail(ctx, GK_EINVAL, "gk_server_start: max_slots must be 1..256");
    if (max_read_len < 1 || max_read_len > GK_MAX_READ_LEN)
        return gk_detail_fail(ctx, GK_EINVAL, "gk_server_start: max_read_len must be 1..512");
    if (mode != GK_SERVER_BATCHED && mode != GK_SERVER_SEQUENTIAL)
        return gk_detail_fail(ctx, GK_EINVAL, "gk_server_start: unknown mode");
    if (device_budget_bytes < (1u << 20))
        return gk_detail_fail(ctx, GK_EINVAL, "gk_server_start: budget below 1 MiB");
    DeviceScope dev(ctx->device);
    gk_server *s = new (std::nothrow) gk_server();
    if (!s)
        return gk_detail_fail(ctx, GK_ENOMEM, "gk_server_start: out of host memory");
    s->ctx = ctx;
    s->mode = mode;
    s->max_slots = max_slots;
    s->max_read_len = max_read_len;
    s->wmax = (max_read_len + 31) / 32;
    s->budget = device_budget_bytes;
    s->arena.init(device_budget_bytes);
    hipError_t e = gk_dmalloc(&s->d_arena, device_budget_bytes);
    s->n_copy = mode == GK_SERVER_BATCHED ? ctx->server_copy_streams : 1u;
    for (uint32_t k = 0; k < s->n_copy && e == hipSuccess; ++k)
        e = hipStreamCreateWithFlags(&s->s_copy[k], hipStreamNonBlocking);
    for (hipStream_t *st : {&s->s_compute, &s->s_d2h})
        if (e == hipSuccess)
            e = hipStreamCreateWithFlags(st, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = gk_dmalloc(&s->d_counters, 2 * sizeof(uint32_t));
    // Every pair takes at least 11 arena bytes, which bounds a tick's pairs.
    const uint64_t resid_cap = device_budget_bytes / 11 + 1;
    if (e == hipSuccess)
        e = gk_dmalloc(&s->d_resid, resid_cap * sizeof(uint32_t));
    if (e == hipSuccess && mode == GK_SERVER_BATCHED) {
        // The tick's persistent launch takes the context's mixed-batch
        // tuning (GK_OPT_MIXED_*, as gk_tune_mixed left it) at start.
        const MixedConfig mc = ctx->mixed;
        const uint32_t ppl = mc.ppl == 2 && s->wmax <= 10 ? 2u : 1u;
        int per_cu = 0;
        e = gkd::mixed_blocks_per_cu(s->wmax, GK_READS_SPLIT, mc.tile, ppl, &per_cu);
        if (per_cu < 1)
            per_cu = 1;
        const uint32_t bpc = mc.blocks_per_cu && (int)mc.blocks_per_cu < per_cu
                                 ? mc.blocks_per_cu
                                 : (uint32_t)per_cu;
        s->part_pairs = ctx->server_part_pairs;
        s->tick_pairs = ctx->server_tick_pairs;
        s->margs.table = nullptr;
        s->margs.tile_counter = s->d_counters;
        s->margs.resid_count = s->d_counters + 1;
        s->margs.resid_list = s->d_resid;
        s->margs.n_tiles = 0;
        s->margs.tile = mc.tile;
        s->margs.ppl = ppl;
        s->margs.sort_e = mc.sort_e;
        s->margs.blocks = bpc * (uint32_t)ctx->cu_count;
        s->margs.resid_blocks = 2u * (uint32_t)ctx->cu_count;
        hipStream_t cap = nullptr;
        if (e == hipSuccess)
            e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
        for (int k = 0; k < 2 && e == hipSuccess; ++k) {
            e = gk_hmalloc(&s->h_table[k], sizeof(gkd::BatchTable));
            if (e == hipSuccess)
                e = gk_dmalloc(&s->d_table[k], sizeof(gkd::BatchTable));
            if (e == hipSuccess)
                e = hipEventCreateWithFlags(&s->tick_done[k], hipEventDisableTiming);
            if (e != hipSuccess)
                break;
            std::memset(s->h_table[k], 0, sizeof(gkd::BatchTable));
            // Tick graph: table copy, reset, persistent kernel, residual pass.
            gkd::MixedArgs x = s->margs;
            x.table = s->d_table[k];
            hipGraph_t g = nullptr;
            e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
            if (e != hipSuccess)
                break;
            hipError_t le = hipMemcpyAsync(s->d_table[k], s->h_table[k], sizeof(gkd::BatchTable),
                                           hipMemcpyHostToDevice, cap);
            if (le == hipSuccess)
                le = gkd::launch_mixed_table(x, s->wmax, GK_READS_SPLIT, cap);
            e = hipStreamEndCapture(cap, &g);
            if (le != hipSuccess)
                e = le;
            if (e == hipSuccess)
                e = hipGraphInstantiate(&s->graph[k], g, nullptr, nullptr, 0);
            if (g)
                (void)hipGraphDestroy(g);
        }
        if (cap)
            (void)hipStreamDestroy(cap);
    }
    if (e != hipSuccess) {
        const int code = e == hipErrorOutOfMemory ? GK_ENOMEM : GK_EDEVICE;
        destroy_server(s);
        return gk_detail_fail(ctx, code,
                              std::string("gk_server_start: ") + hipGetErrorName(e));
    }
    gk_detail_log(ctx, "gk_server_start: %s, %llu device bytes, %u slots, words per mask up "
                  "to %u, %u copy streams; ticks of up to %llu pairs, parts of up to %llu, "
                  "tile %u", mode == GK_SERVER_BATCHED ? "batched" : "sequential",
                  (unsigned long long)device_budget_bytes, max_slots, s->wmax, s->n_copy,
                  (unsigned long long)s->tick_pairs, (unsigned long long)s->part_pairs,
                  s->margs.tile);
    s->loader = std::thread(loader_main, s);
    if (mode == GK_SERVER_BATCHED) {
        s->scheduler = std::thread(scheduler_main, s);
        s->completer = std::thread(completer_main, s);
    }
    *out = s;
    return GK_OK;
}

int gk_server_submit(gk_server *s, const gk_request *r, uint64_t *ticket)
{
    if (!s || !r || !ticket)
        return GK_EINVAL;
    if (r->n_reads == 0 && r->n_pairs > 0)
        return GK_EINVAL;
    if (r->n_reads >= (1u << 30) || r->n_pairs >= (1ull << 30) || r->e > 255)
        return GK_EINVAL;
    if ((r->n_reads && (!r->reads || !r->read_off)) ||
        (r->n_pairs && (!r->cand_pos || !r->accept || !r->est)))
        return GK_EINVAL;
    Req *q = new (std::nothrow) Req();
    if (!q)
        return GK_ENOMEM;
    q->r = *r;
    q->t_submit = r->t_arrival_us ? r->t_arrival_us : now_us();
    if (r->n_reads)
        plan(q);
    if (q->max_len > s->max_read_len) {
        delete q;
        return GK_ERANGE;
    }
    if (q->footprint > s->budget) {
        delete q;
        return GK_ERANGE;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) {
        delete q;
        return GK_EDEVICE;
    }
    if (hipEventCreateWithFlags(&q->ready, hipEventDisableTiming) != hipSuccess) {
        delete q;
        return GK_EDEVICE;
    }
    q->ticket = s->next_ticket++;
    s->reqs[q->ticket] = q;
    if (r->n_pairs == 0) {
        q->t_admit = q->t_submit;    // nothing to admit: done at once
        finish(s, q, GK_OK);
    } else {
        s->pending.push_back(q);
        s->cv.notify_all();
    }
    *ticket = q->ticket;
    return GK_OK;
}

int gk_server_wait(gk_server *s, uint64_t ticket, int64_t timeout_us, gk_request_stats *stats)
{
    if (!s)
        return GK_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end())
        return GK_EINVAL;
    Req *q = it->second;
    auto done = [&] { return q->done; };
    if (timeout_us < 0) {
        s->cv.wait(lk, done);
    } else if (!s->cv.wait_for(lk, std::chrono::microseconds(timeout_us), done)) {
        return GK_ETIMEOUT;
    }
    if (stats) {
        stats->status = q->status;
        stats->n_pairs = q->r.n_pairs;
        stats->t_submit_us = q->t_submit;
        stats->t_admit_us = q->t_admit;
        stats->t_done_us = q->t_done;
    }
    const int st = q->status;
    s->reqs.erase(it);
    lk.unlock();
    if (q->ready) {
        DeviceScope dev(s->ctx->device);
        (void)hipEventDestroy(q->ready);
    }
    delete q;
    return st;
}

int gk_server_counters(gk_server *s, uint64_t *ticks, uint64_t *max_requests_per_tick,
                       uint64_t *pairs_done)
{
    if (!s)
        return GK_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (ticks)
        *ticks = s->ticks;
    if (max_requests_per_tick)
        *max_requests_per_tick = s->tick_req_max;
    if (pairs_done)
        *pairs_done = s->pairs_done;
    return GK_OK;
}

int gk_server_tick_log(gk_server *s, gk_tick_record *out, uint64_t cap, uint64_t *n_total)
{
    if (!s || (cap && !out))
        return GK_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    const uint64_t n = s->tick_log.size();
    if (n_total)
        *n_total = n;
    if (cap)
        std::memcpy(out, s->tick_log.data(), (n < cap ? n : cap) * sizeof(gk_tick_record));
    return GK_OK;
}

int gk_server_stop(gk_server *s)
{
    if (!s)
        return GK_EINVAL;
    {
        // Requests not admitted yet are cancelled; admitted ones finish.
        std::unique_lock<std::mutex> lk(s->mu);
        for (auto *q : s->pending)
            finish(s, q, GK_ECANCELED);
        s->pending.clear();
        s->cv.notify_all();
        s->cv.wait(lk, [&] {
            return s->stopping ||
                   (s->ready.empty() && s->inflight.empty() && s->slots_used == 0);
        });
        s->stopping = true;
        s->cv.notify_all();
    }
    if (s->loader.joinable())
        s->loader.join();
    if (s->scheduler.joinable())
        s->scheduler.join();
    if (s->completer.joinable())
        s->completer.join();
    const int st = s->err.empty() ? GK_OK : GK_EDEVICE;
    destroy_server(s);
    return st;
}

int64_t gk_clock_us(void) { return now_us(); }

// For tests of the error paths (no GPU fault): the server's load number
// `load_at` (counted from 1 in admission order), or its completed tick number
// `tick_at`, fails as a failed HIP call would; 0 leaves that point alone.
// Call before submitting requests.
int gk_detail_server_inject_failure(gk_server *s, uint64_t load_at, uint64_t tick_at)
{
    if (!s)
        return GK_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    s->fail_load_at = load_at;
    s->fail_tick_at = tick_at;
    return GK_OK;
}

}  // extern "C"

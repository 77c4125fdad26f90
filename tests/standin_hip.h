// Stand-in HIP runtime for CPU checks of the library's host logic (a source
// file built as host C++ against the HIP headers, without the HIP runtime):
// every stream has a worker thread that runs its operations in order (copies
// are memcpy; an event fires when its stream reaches it; a captured graph
// replays its recorded operations), and device memory is host memory.
// Included by exactly one translation unit of a check program.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "gk_internal.h"

// ---- stand-in HIP runtime ---------------------------------------------------

namespace {

struct Op {
    std::function<void()> fn;
};

// Up to this many microseconds of sleep before each stream operation, at
// random, so that a missing wait between streams shows as wrong results.
std::atomic<int> g_jitter_us{0};

// Device bytes allocated and not yet freed, and their peak.
std::mutex g_alloc_mu;
std::map<void *, size_t> g_alloc_live;
size_t g_alloc_bytes = 0, g_alloc_peak = 0;

}  // namespace

struct ihipStream_t {
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Op> q;
    uint64_t enqueued = 0, done = 0;
    bool stop = false;
    bool capturing = false;
    std::vector<Op> captured;
    std::thread worker;

    ihipStream_t()
    {
        worker = std::thread([this] {
            std::minstd_rand rng((uint32_t)(uintptr_t)this);
            std::unique_lock<std::mutex> lk(mu);
            while (true) {
                cv.wait(lk, [&] { return stop || !q.empty(); });
                if (q.empty() && stop)
                    return;
                Op op = std::move(q.front());
                q.pop_front();
                lk.unlock();
                const int jitter = g_jitter_us.load();
                if (jitter > 0)
                    std::this_thread::sleep_for(std::chrono::microseconds(rng() % jitter));
                op.fn();
                lk.lock();
                done++;
                cv.notify_all();
            }
        });
    }
    ~ihipStream_t()
    {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
            cv.notify_all();
        }
        worker.join();
    }
    void enqueue(std::function<void()> fn)
    {
        std::lock_guard<std::mutex> lk(mu);
        if (capturing) {
            captured.push_back(Op{std::move(fn)});
            return;
        }
        q.push_back(Op{std::move(fn)});
        enqueued++;
        cv.notify_all();
    }
    void sync()
    {
        std::unique_lock<std::mutex> lk(mu);
        const uint64_t target = enqueued;
        cv.wait(lk, [&] { return done >= target; });
    }
};

// An event's state outlives its handle while stream operations still refer
// to it (as the runtime allows destroying an event that is still pending).
struct EventState {
    std::mutex mu;
    std::condition_variable cv;
    uint64_t recorded = 0, fired = 0;   // generations
};

struct ihipEvent_t {
    std::shared_ptr<EventState> st = std::make_shared<EventState>();
};

struct ihipGraph {
    std::vector<Op> ops;
};

struct hipGraphExec {
    std::vector<Op> ops;
};

namespace {

void event_wait(const std::shared_ptr<EventState> &ev, uint64_t gen)
{
    std::unique_lock<std::mutex> lk(ev->mu);
    ev->cv.wait(lk, [&] { return ev->fired >= gen; });
}

}  // namespace

extern "C" {

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int)
{
    *s = new ihipStream_t();
    return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t s)
{
    delete s;
    return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t s)
{
    s->sync();
    return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t *ev, unsigned int)
{
    *ev = new ihipEvent_t();
    return hipSuccess;
}

hipError_t hipEventDestroy(hipEvent_t ev)
{
    delete ev;
    return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t ev, hipStream_t s)
{
    std::shared_ptr<EventState> st = ev->st;
    uint64_t gen;
    {
        std::lock_guard<std::mutex> lk(st->mu);
        gen = ++st->recorded;
    }
    s->enqueue([st, gen] {
        std::lock_guard<std::mutex> lk(st->mu);
        if (st->fired < gen)
            st->fired = gen;
        st->cv.notify_all();
    });
    return hipSuccess;
}

hipError_t hipEventSynchronize(hipEvent_t ev)
{
    uint64_t gen;
    {
        std::lock_guard<std::mutex> lk(ev->st->mu);
        gen = ev->st->recorded;
    }
    event_wait(ev->st, gen);
    return hipSuccess;
}

hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t ev, unsigned int)
{
    std::shared_ptr<EventState> st = ev->st;
    uint64_t gen;
    {
        std::lock_guard<std::mutex> lk(st->mu);
        gen = st->recorded;
    }
    s->enqueue([st, gen] { event_wait(st, gen); });
    return hipSuccess;
}

hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind, hipStream_t s)
{
    s->enqueue([dst, src, n] { std::memcpy(dst, src, n); });
    return hipSuccess;
}

hipError_t hipMemsetAsync(void *dst, int v, size_t n, hipStream_t s)
{
    s->enqueue([dst, v, n] { std::memset(dst, v, n); });
    return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode)
{
    std::lock_guard<std::mutex> lk(s->mu);
    s->capturing = true;
    s->captured.clear();
    return hipSuccess;
}

hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g)
{
    std::lock_guard<std::mutex> lk(s->mu);
    s->capturing = false;
    auto *graph = new ihipGraph();
    graph->ops = std::move(s->captured);
    s->captured.clear();
    *g = graph;
    return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t *exec, hipGraph_t g, hipGraphNode_t *, char *,
                               size_t)
{
    auto *x = new hipGraphExec();
    x->ops = g->ops;
    *exec = x;
    return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t g)
{
    delete g;
    return hipSuccess;
}

hipError_t hipGraphExecDestroy(hipGraphExec_t x)
{
    delete x;
    return hipSuccess;
}

hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s)
{
    for (const Op &op : x->ops)
        s->enqueue(op.fn);
    return hipSuccess;
}

hipError_t hipFree(void *p)
{
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        auto it = g_alloc_live.find(p);
        if (it != g_alloc_live.end()) {
            g_alloc_bytes -= it->second;
            g_alloc_live.erase(it);
        }
    }
    std::free(p);
    return hipSuccess;
}

hipError_t hipHostFree(void *p)
{
    std::free(p);
    return hipSuccess;
}

hipError_t hipSetDevice(int) { return hipSuccess; }

hipError_t hipGetDevice(int *d)
{
    *d = 0;
    return hipSuccess;
}

const char *hipGetErrorName(hipError_t e)
{
    return e == hipSuccess ? "hipSuccess" : "hipError (stand-in)";
}

const char *hipGetErrorString(hipError_t e)
{
    return e == hipSuccess ? "no error" : "stand-in error";
}

}  // extern "C"

namespace {

void *zalloc(size_t bytes)
{
    const size_t n = (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
    void *p = std::aligned_alloc(256, n);
    if (p)
        std::memset(p, 0, n);
    return p;
}

}  // namespace

hipError_t gk_detail_device_alloc(void **p, size_t bytes)
{
    *p = zalloc(bytes);
    if (!*p)
        return hipErrorOutOfMemory;
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc_live[*p] = bytes;
    g_alloc_bytes += bytes;
    g_alloc_peak = std::max(g_alloc_peak, g_alloc_bytes);
    return hipSuccess;
}

hipError_t gk_detail_pinned_alloc(void **p, size_t bytes)
{
    *p = zalloc(bytes);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}

// The library's log line (defined with the entry points, which a check
// program does not build).
void gk_detail_log(const gk_ctx *ctx, const char *fmt, ...)
{
    if (!ctx || !ctx->log)
        return;
    va_list ap;
    va_start(ap, fmt);
    std::fputs("[gk] ", stderr);
    std::vfprintf(stderr, fmt, ap);
    std::fputs("\n", stderr);
    va_end(ap);
}

// Host side of libgk: context, resident reference, argument checks, launches.
#include <algorithm>
#include <atomic>
#include <cerrno>
#include <cstdarg>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <new>
#include <sstream>
#include <string>

#include "gk_internal.h"
#include "gk_trace.h"
#include "gk_reference.h"
#include "gk_verify.h"

namespace {

thread_local std::string g_create_error;

using DeviceGuard = DeviceScope;

int fail(gk_ctx *ctx, int code, const std::string &msg) { return gk_detail_fail(ctx, code, msg); }

int hip_fail(gk_ctx *ctx, hipError_t e, const char *what)
{
    std::string msg = std::string(what) + ": " + hipGetErrorName(e) + " (" +
                      hipGetErrorString(e) + ")";
    return fail(ctx, e == hipErrorOutOfMemory ? GK_ENOMEM : GK_EDEVICE, msg);
}

void free_reference(gk_ctx *ctx)
{
    if (ctx->ref_planes)
        (void)hipFree(ctx->ref_planes);
    if (ctx->ref_unk)
        (void)hipFree(ctx->ref_unk);
    if (ctx->ref_planes_b)
        (void)hipFree(ctx->ref_planes_b);
    ctx->ref_planes_b = nullptr;
    if (ctx->ref_unk_lines)
        (void)hipFree(ctx->ref_unk_lines);
    ctx->ref_unk_lines = nullptr;
    ctx->ref_planes = nullptr;
    ctx->ref_unk = nullptr;
    ctx->ref_len = ctx->ref_words = ctx->ref_unknown = 0;
}

// Derived views of a loaded reference: the shifted copy of the planes (see
// gkd::REF_SHIFT_WORDS) and the one-bit-per-line summary of the unknown plane,
// which lets a pair skip the unknown-plane gather when its window's lines
// hold no unknown base.
hipError_t finish_reference(gk_ctx *ctx, uint64_t words, uint64_t alloc_words,
                            uint64_t unknown)
{
    const uint64_t k = gkd::REF_SHIFT_WORDS;
    hipError_t e = gk_dmalloc(&ctx->ref_planes_b, alloc_words * sizeof(uint2));
    if (e == hipSuccess)
        e = hipMemset(ctx->ref_planes_b + (alloc_words - k), 0, k * sizeof(uint2));
    if (e == hipSuccess)
        e = hipMemcpy(ctx->ref_planes_b, ctx->ref_planes + k, (alloc_words - k) * sizeof(uint2),
                      hipMemcpyDeviceToDevice);
    const uint64_t line_words = ((words + gkd::LINE_WORDS - 1) / gkd::LINE_WORDS + 63) / 64 + 1;
    if (e == hipSuccess)
        e = gk_dmalloc(&ctx->ref_unk_lines, line_words * sizeof(unsigned long long));
    if (e == hipSuccess)
        e = hipMemset(ctx->ref_unk_lines, 0, line_words * sizeof(unsigned long long));
    if (e == hipSuccess && unknown > 0)
        e = gkd::launch_unknown_lines(ctx->ref_unk, words, ctx->ref_unk_lines, nullptr);
    if (e == hipSuccess)
        e = hipDeviceSynchronize();
    return e;
}

// Scratch of gk_filter_mixed_noalloc: the tile counter and the residual
// count (words 0 and 1), then, from word NOALLOC_LIST_WORD, the residual
// list of up to GK_NOALLOC_MAX_PAIRS pair indices.  A file-scope device
// array, so the entry point allocates nothing; every device holds its own
// copy until the process ends.  Host code never uses the name itself: its
// device address is taken once per device (scratch_setup, from gk_create)
// and kept in g_scratch.
}  // namespace

namespace gkd {
constexpr uint32_t NOALLOC_LIST_WORD = 64;
__device__ __align__(256) uint32_t scratch[NOALLOC_LIST_WORD + GK_NOALLOC_MAX_PAIRS];
}  // namespace gkd

namespace {

constexpr int MAX_DEVICES = 256;
std::mutex g_scratch_mu;
uint32_t *g_scratch[MAX_DEVICES] = {};

// With `device` current: its address of the scratch array, once per device.
hipError_t scratch_setup(int device)
{
    if (device < 0 || device >= MAX_DEVICES)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[device])
        return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(gkd::scratch));
    if (e != hipSuccess)
        return e;
    if (!p)
        return hipErrorInvalidSymbol;
    g_scratch[device] = static_cast<uint32_t *>(p);
    return hipSuccess;
}

std::atomic<uint64_t> g_fail_alloc_at{0};   // 0: allocations are never failed

// Whether this allocation is the one gk_detail_fail_alloc asked to fail.
bool take_injected_failure()
{
    uint64_t left = g_fail_alloc_at.load();
    while (left != 0)
        if (g_fail_alloc_at.compare_exchange_weak(left, left - 1))
            return left == 1;
    return false;
}

uint32_t *scratch_of(int device)
{
    if (device < 0 || device >= MAX_DEVICES)
        return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch[device];
}

}  // namespace

hipError_t gk_detail_device_alloc(void **p, size_t bytes)
{
    if (take_injected_failure()) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

hipError_t gk_detail_pinned_alloc(void **p, size_t bytes)
{
    if (take_injected_failure()) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipHostMalloc(p, bytes, hipHostMallocDefault);
}

void gk_detail_log(const gk_ctx *ctx, const char *fmt, ...)
{
    if (!ctx || !ctx->log)
        return;
    char line[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(line, sizeof line, fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "[gk] %s\n", line);
}

extern "C" {

// Test hook (not part of the public header): the nth device or pinned-host
// allocation the library makes from now on, in any context, reports
// hipErrorOutOfMemory and allocates nothing; 0 cancels a pending one.
int gk_detail_fail_alloc(uint64_t nth)
{
    g_fail_alloc_at.store(nth);
    return GK_OK;
}

namespace {

// Options a context takes from the environment at creation: GK_<name> for
// option GK_OPT_<name>, a decimal integer in the option's range.
constexpr struct {
    const char *var;
    int option;
} ENV_OPTIONS[] = {
    {"GK_PAIRS_PER_LANE", GK_OPT_PAIRS_PER_LANE},
    {"GK_MIXED_TILE", GK_OPT_MIXED_TILE},
    {"GK_MIXED_PAIRS_PER_LANE", GK_OPT_MIXED_PAIRS_PER_LANE},
    {"GK_MIXED_SORT_E", GK_OPT_MIXED_SORT_E},
    {"GK_MIXED_BLOCKS_PER_CU", GK_OPT_MIXED_BLOCKS_PER_CU},
    {"GK_MIXED_GRAPH", GK_OPT_MIXED_GRAPH},
    {"GK_HOST_ENCODE_THREADS", GK_OPT_HOST_ENCODE_THREADS},
    {"GK_SERVER_PART_PAIRS", GK_OPT_SERVER_PART_PAIRS},
    {"GK_SERVER_TICK_PAIRS", GK_OPT_SERVER_TICK_PAIRS},
    {"GK_HOST_CHUNK_PAIRS", GK_OPT_HOST_CHUNK_PAIRS},
    {"GK_SERVER_COPY_STREAMS", GK_OPT_SERVER_COPY_STREAMS},
};

// GK_FAULT_INJECT=alloc:N arms the allocation-failure hook once per process
// (the N-th device or pinned allocation from the first gk_create on fails).
std::mutex g_fault_env_mu;
bool g_fault_env_done = false;

int apply_env_flags(gk_ctx *ctx)
{
    if (const char *v = std::getenv("GK_LOG")) {
        if (std::strcmp(v, "0") != 0 && std::strcmp(v, "1") != 0)
            return fail(ctx, GK_EINVAL, std::string("gk_create: GK_LOG='") + v +
                                            "' must be 0 or 1");
        ctx->log = v[0] == '1';
    }
    if (const char *v = std::getenv("GK_AUTOTUNE")) {
        if (!std::strcmp(v, "use"))
            ctx->autotune = AUTOTUNE_USE;
        else if (!std::strcmp(v, "refresh"))
            ctx->autotune = AUTOTUNE_REFRESH;
        else if (!std::strcmp(v, "off"))
            ctx->autotune = AUTOTUNE_OFF;
        else
            return fail(ctx, GK_EINVAL, std::string("gk_create: GK_AUTOTUNE='") + v +
                                            "' must be use, refresh or off");
    }
    return GK_OK;
}

// Parses GK_FAULT_INJECT before gk_create allocates anything; returns a
// message for a malformed value, else "".
std::string arm_fault_from_env()
{
    const char *v = std::getenv("GK_FAULT_INJECT");
    if (!v)
        return "";
    char *end = nullptr;
    errno = 0;
    const unsigned long long n =
        std::strncmp(v, "alloc:", 6) == 0 ? std::strtoull(v + 6, &end, 10) : 0ull;
    if (n == 0 || errno != 0 || !end || *end != '\0' || v[6] == '-')
        return std::string("gk_create: GK_FAULT_INJECT='") + v + "' must be alloc:N with N >= 1";
    std::lock_guard<std::mutex> lk(g_fault_env_mu);
    if (!g_fault_env_done) {
        g_fail_alloc_at.store(n);
        g_fault_env_done = true;
    }
    return "";
}

int apply_env_options(gk_ctx *ctx)
{
    for (const auto &o : ENV_OPTIONS) {
        const char *v = std::getenv(o.var);
        if (!v)
            continue;
        char *end = nullptr;
        errno = 0;
        const long long x = std::strtoll(v, &end, 10);
        if (errno != 0 || end == v || *end != '\0')
            return fail(ctx, GK_EINVAL,
                        std::string("gk_create: ") + o.var + "='" + v + "' is not an integer");
        const int st = gk_set_option(ctx, o.option, (int64_t)x);
        if (st != GK_OK)
            return fail(ctx, st, std::string("gk_create: ") + o.var + ": " + ctx->err);
    }
    return GK_OK;
}

}  // namespace

int gk_create(int device, gk_ctx **out)
{
    if (!out) {
        g_create_error = "gk_create: out is NULL";
        return GK_EINVAL;
    }
    *out = nullptr;
    const std::string fault_err = arm_fault_from_env();
    if (!fault_err.empty()) {
        g_create_error = fault_err;
        return GK_EINVAL;
    }
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || device < 0 || device >= count) {
        g_create_error = "gk_create: no HIP device " + std::to_string(device) + " (" +
                         std::to_string(count) + " visible)";
        return e != hipSuccess ? GK_EDEVICE : GK_EINVAL;
    }
    gk_ctx *ctx = new (std::nothrow) gk_ctx();
    if (!ctx) {
        g_create_error = "gk_create: out of host memory";
        return GK_ENOMEM;
    }
    ctx->device = device;
    DeviceGuard g(device);
    if (!g.ok) {
        delete ctx;
        g_create_error = "gk_create: hipSetDevice failed";
        return GK_EDEVICE;
    }
    e = hipDeviceGetAttribute(&ctx->cu_count, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess || ctx->cu_count < 1) {
        delete ctx;
        g_create_error = "gk_create: cannot read the compute unit count";
        return GK_EDEVICE;
    }
    e = gk_dmalloc(&ctx->d_counter, sizeof(unsigned long long));
    if (e != hipSuccess) {
        delete ctx;
        g_create_error = std::string("gk_create: hipMalloc: ") + hipGetErrorName(e);
        return e == hipErrorOutOfMemory ? GK_ENOMEM : GK_EDEVICE;
    }
    e = scratch_setup(device);
    if (e != hipSuccess) {
        (void)hipFree(ctx->d_counter);
        delete ctx;
        g_create_error = std::string("gk_create: device scratch address: ") +
                         hipGetErrorName(e);
        return GK_EDEVICE;
    }
    int st = apply_env_options(ctx);
    if (st == GK_OK)
        st = apply_env_flags(ctx);
    if (st != GK_OK) {
        g_create_error = ctx->err;
        gk_destroy(ctx);
        return st;
    }
    g_create_error.clear();
    *out = ctx;
    return GK_OK;
}

void gk_destroy(gk_ctx *ctx)
{
    if (!ctx)
        return;
    {
        DeviceGuard g(ctx->device);
        free_reference(ctx);
        if (ctx->d_counter)
            (void)hipFree(ctx->d_counter);
        if (ctx->graph_exec)
            (void)hipGraphExecDestroy(ctx->graph_exec);
        if (ctx->d_mixed_counters)
            (void)hipFree(ctx->d_mixed_counters);
        if (ctx->d_resid)
            (void)hipFree(ctx->d_resid);
        if (ctx->capture_stream)
            (void)hipStreamDestroy(ctx->capture_stream);
        if (ctx->d_table)
            (void)hipFree(ctx->d_table);
        for (int k = 0; k < gk_ctx::TABLE_RING; ++k) {
            if (ctx->h_table[k])
                (void)hipHostFree(ctx->h_table[k]);
            if (ctx->table_ev[k])
                (void)hipEventDestroy(ctx->table_ev[k]);
        }
        gk_detail_free_host_pipe(ctx);
        if (ctx->d_verify_list)
            (void)hipFree(ctx->d_verify_list);
        if (ctx->d_verify_count)
            (void)hipFree(ctx->d_verify_count);
        if (ctx->d_reads_rm)
            (void)hipFree(ctx->d_reads_rm);
    }
    delete ctx;
}

const char *gk_last_error(const gk_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

int gk_load_reference(gk_ctx *ctx, const char *ascii, uint64_t len)
{
    gkd::TraceRange trace("gk_load_reference");
    if (!ctx)
        return GK_EINVAL;
    if (!ascii || len == 0)
        return fail(ctx, GK_EINVAL, "gk_load_reference: empty or NULL reference");
    if (len > GK_MAX_REF_LEN)
        return fail(ctx, GK_ERANGE, "gk_load_reference: reference longer than 2^32-1 bases");
    DeviceGuard g(ctx->device);
    if (!g.ok)
        return fail(ctx, GK_EDEVICE, "gk_load_reference: hipSetDevice failed");
    free_reference(ctx);

    const uint64_t words = (len + 31) / 32;
    const uint64_t alloc_words = words + gkd::REF_PAD_WORDS;
    hipError_t e = gk_dmalloc(&ctx->ref_planes, alloc_words * sizeof(uint2));
    if (e != hipSuccess)
        return free_reference(ctx), hip_fail(ctx, e, "gk_load_reference: hipMalloc planes");
    e = gk_dmalloc(&ctx->ref_unk, alloc_words * sizeof(uint32_t));
    if (e != hipSuccess)
        return free_reference(ctx), hip_fail(ctx, e, "gk_load_reference: hipMalloc unknown");
    e = hipMemset(ctx->ref_planes, 0, alloc_words * sizeof(uint2));
    if (e == hipSuccess)
        e = hipMemset(ctx->ref_unk, 0, alloc_words * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipMemset(ctx->d_counter, 0, sizeof(unsigned long long));
    if (e != hipSuccess)
        return free_reference(ctx), hip_fail(ctx, e, "gk_load_reference: hipMemset");

    // Stage the ASCII through a device buffer in chunks of `step` bases, a
    // multiple of 32 and at least 32 (len >= 1), and pack each chunk on the GPU.
    const uint64_t step = std::min<uint64_t>((len + 31) & ~uint64_t(31), 256ull << 20);
    uint8_t *stage = nullptr;
    e = gk_dmalloc(&stage, step);
    if (e != hipSuccess)
        return free_reference(ctx), hip_fail(ctx, e, "gk_load_reference: hipMalloc staging");
    for (uint64_t first = 0; first < len && e == hipSuccess; first += step) {
        const uint64_t n = std::min<uint64_t>(step, len - first);
        e = hipMemcpy(stage, ascii + first, n, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = gkd::launch_pack_reference(stage, first, n, ctx->ref_planes, ctx->ref_unk,
                                           ctx->d_counter, nullptr);
        if (e == hipSuccess)
            e = hipDeviceSynchronize();
    }
    unsigned long long unknown = 0;
    if (e == hipSuccess)
        e = hipMemcpy(&unknown, ctx->d_counter, sizeof unknown, hipMemcpyDeviceToHost);
    (void)hipFree(stage);
    if (e == hipSuccess)
        e = finish_reference(ctx, words, alloc_words, unknown);
    if (e != hipSuccess)
        return free_reference(ctx), hip_fail(ctx, e, "gk_load_reference: pack");
    ctx->ref_len = len;
    ctx->ref_words = words;
    ctx->ref_unknown = unknown;
    ctx->err.clear();
    return GK_OK;
}

int gk_load_reference_2bit(gk_ctx *ctx, const uint32_t *packed, uint64_t len, uint32_t layout,
                           const uint64_t *n_runs, uint64_t n_n_runs)
{
    gkd::TraceRange trace("gk_load_reference_2bit");
    if (!ctx)
        return GK_EINVAL;
    if (!packed || len == 0)
        return fail(ctx, GK_EINVAL, "gk_load_reference_2bit: empty or NULL reference");
    if (len > GK_MAX_REF_LEN)
        return fail(ctx, GK_ERANGE, "gk_load_reference_2bit: reference longer than 2^32-1 bases");
    if (layout != GK_READS_SPLIT && layout != GK_READS_INTERLEAVED)
        return fail(ctx, GK_EINVAL, "gk_load_reference_2bit: unknown layout");
    if (n_n_runs > 0 && !n_runs)
        return fail(ctx, GK_EINVAL, "gk_load_reference_2bit: n_runs is NULL");
    if (n_n_runs > (1ull << 40))
        return fail(ctx, GK_EINVAL, "gk_load_reference_2bit: too many runs");
    for (uint64_t r = 0; r < n_n_runs; ++r) {
        const uint64_t s = n_runs[2 * r], l = n_runs[2 * r + 1];
        if (l > 0 && (s >= len || l > len - s))
            return fail(ctx, GK_EINVAL, "gk_load_reference_2bit: run " + std::to_string(r) +
                                            " reaches past the reference end");
    }
    DeviceGuard g(ctx->device);
    if (!g.ok)
        return fail(ctx, GK_EDEVICE, "gk_load_reference_2bit: hipSetDevice failed");
    free_reference(ctx);

    const uint64_t words = (len + 31) / 32;
    const uint64_t alloc_words = words + gkd::REF_PAD_WORDS;
    hipError_t e = gk_dmalloc(&ctx->ref_planes, alloc_words * sizeof(uint2));
    if (e != hipSuccess)
        return free_reference(ctx), hip_fail(ctx, e, "gk_load_reference_2bit: hipMalloc planes");
    e = gk_dmalloc(&ctx->ref_unk, alloc_words * sizeof(uint32_t));
    if (e != hipSuccess)
        return free_reference(ctx), hip_fail(ctx, e, "gk_load_reference_2bit: hipMalloc unknown");
    e = hipMemset(ctx->ref_planes, 0, alloc_words * sizeof(uint2));
    if (e == hipSuccess)
        e = hipMemset(ctx->ref_unk, 0, alloc_words * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipMemset(ctx->d_counter, 0, sizeof(unsigned long long));
    if (e != hipSuccess)
        return free_reference(ctx), hip_fail(ctx, e, "gk_load_reference_2bit: hipMemset");

    // Stage the words in chunks of `step` bases (a multiple of 32, at most
    // 2^30 bases = 256 MiB of words) and unpack each chunk on the GPU.
    const uint64_t step = std::min<uint64_t>((len + 31) & ~uint64_t(31), 1ull << 30);
    uint32_t *stage = nullptr;
    e = gk_dmalloc(&stage, step / 16 * sizeof(uint32_t));
    if (e != hipSuccess)
        return free_reference(ctx), hip_fail(ctx, e, "gk_load_reference_2bit: hipMalloc staging");
    for (uint64_t first = 0; first < len && e == hipSuccess; first += step) {
        const uint64_t n = std::min<uint64_t>(step, len - first);
        e = hipMemcpy(stage, packed + first / 16, (n + 15) / 16 * sizeof(uint32_t),
                      hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = gkd::launch_unpack_reference(stage, first, n, layout, ctx->ref_planes, nullptr);
        if (e == hipSuccess)
            e = hipDeviceSynchronize();
    }
    (void)hipFree(stage);
    uint64_t *d_runs = nullptr;
    if (e == hipSuccess && n_n_runs > 0) {
        e = gk_dmalloc(&d_runs, n_n_runs * 2 * sizeof(uint64_t));
        if (e == hipSuccess)
            e = hipMemcpy(d_runs, n_runs, n_n_runs * 2 * sizeof(uint64_t), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = gkd::launch_mark_runs(d_runs, n_n_runs, ctx->ref_unk, nullptr);
    }
    if (e == hipSuccess && n_n_runs > 0)
        e = gkd::launch_count_unknown(ctx->ref_unk, words, ctx->d_counter, nullptr);
    if (e == hipSuccess)
        e = hipDeviceSynchronize();
    if (d_runs)
        (void)hipFree(d_runs);
    unsigned long long unknown = 0;
    if (e == hipSuccess)
        e = hipMemcpy(&unknown, ctx->d_counter, sizeof unknown, hipMemcpyDeviceToHost);
    if (e == hipSuccess)
        e = finish_reference(ctx, words, alloc_words, unknown);
    if (e != hipSuccess)
        return free_reference(ctx), hip_fail(ctx, e, "gk_load_reference_2bit: unpack");
    ctx->ref_len = len;
    ctx->ref_words = words;
    ctx->ref_unknown = unknown;
    ctx->err.clear();
    return GK_OK;
}

int gk_reference_info(const gk_ctx *ctx, uint64_t *len, uint64_t *n_unknown)
{
    if (!ctx)
        return GK_EINVAL;
    if (!ctx->ref_planes)
        return GK_ENOREF;
    if (len)
        *len = ctx->ref_len;
    if (n_unknown)
        *n_unknown = ctx->ref_unknown;
    return GK_OK;
}

int gk_encode_reads(gk_ctx *ctx, const uint8_t *ascii, const uint64_t *read_off, uint32_t n_reads,
                    uint32_t pitch, uint32_t rows, uint32_t layout, uint32_t *packed_out,
                    uint16_t *len_out, uint8_t *has_n_out, void *stream)
{
    gkd::TraceRange trace("gk_encode_reads");
    if (!ctx)
        return GK_EINVAL;
    if (n_reads == 0)
        return GK_OK;
    if (!ascii || !read_off || !packed_out || !len_out)
        return fail(ctx, GK_EINVAL, "gk_encode_reads: NULL buffer");
    if (pitch < n_reads)
        return fail(ctx, GK_EINVAL, "gk_encode_reads: pitch < n_reads");
    if (n_reads >= (1u << 30) || pitch >= (1u << 30))
        return fail(ctx, GK_EINVAL, "gk_encode_reads: n_reads and pitch must be below 2^30");
    if (rows < 1 || rows > 32)
        return fail(ctx, GK_EINVAL, "gk_encode_reads: rows must be 1..32");
    if (layout != GK_READS_SPLIT && layout != GK_READS_INTERLEAVED)
        return fail(ctx, GK_EINVAL, "gk_encode_reads: unknown layout");
    DeviceGuard g(ctx->device);
    if (!g.ok)
        return fail(ctx, GK_EDEVICE, "gk_encode_reads: hipSetDevice failed");
    hipError_t e = gkd::launch_encode_reads(ascii, read_off, n_reads, pitch, rows, layout,
                                            packed_out, len_out, has_n_out, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "gk_encode_reads: launch");
    return GK_OK;
}

}  // extern "C"

namespace {

// Checks a batch (nothing launched on failure) and fills the kernel
// arguments.  Returns GK_OK, a GK_E* code, or 1 for an empty batch.
int prepare_batch(gk_ctx *ctx, const gk_batch *b, const char *who, gkd::FilterArgs &a)
{
    const std::string w(who);
    if (!b)
        return fail(ctx, GK_EINVAL, w + ": batch is NULL");
    if (!ctx->ref_planes)
        return fail(ctx, GK_ENOREF, w + ": no reference loaded");
    if (b->max_read_len < 1 || b->max_read_len > GK_MAX_READ_LEN)
        return fail(ctx, GK_EINVAL, w + ": max_read_len must be 1..512");
    if (b->e_uniform > 255)
        return fail(ctx, GK_EINVAL, w + ": e_uniform must be 0..255");
    if (b->pitch < b->n_reads)
        return fail(ctx, GK_EINVAL, w + ": pitch < n_reads");
    if (b->n_reads >= (1u << 30) || b->pitch >= (1u << 30))
        return fail(ctx, GK_EINVAL, w + ": n_reads and pitch must be below 2^30");
    if (b->read_layout != GK_READS_SPLIT && b->read_layout != GK_READS_INTERLEAVED)
        return fail(ctx, GK_EINVAL, w + ": unknown read_layout");
    if (b->flags & ~(GK_FLAG_NO_REFINE | GK_FLAG_HAMMING_FASTPATH))
        return fail(ctx, GK_EINVAL, w + ": unknown flags");
    if (b->n_pairs == 0)
        return 1;
    if (b->n_pairs >= (1ull << 38))
        return fail(ctx, GK_ERANGE, w + ": n_pairs must be below 2^38");
    if (!b->cand_pos || !b->accept || !b->est)
        return fail(ctx, GK_EINVAL, w + ": NULL pair or output buffer");
    if (b->n_reads > 0 && (!b->reads || !b->read_len))
        return fail(ctx, GK_EINVAL, w + ": NULL read buffer");
    a.flags = b->flags;
    a.ref_planes = ctx->ref_planes;
    a.ref_planes_b = ctx->ref_planes_b;
    a.ref_unk = ctx->ref_unk;
    a.ref_unk_lines = ctx->ref_unk_lines;
    a.ref_len = ctx->ref_len;
    a.ref_has_unknown = ctx->ref_unknown > 0;
    a.n_reads = b->n_reads;
    a.pitch = b->pitch;
    a.e_uniform = b->e_uniform;
    a.max_read_len = b->max_read_len;
    a.rows = (b->max_read_len + 15) / 16;
    a.reads = b->reads;
    a.read_len = b->read_len;
    a.read_has_n = b->read_has_n;
    a.pair_read = b->pair_read;
    a.cand_pos = b->cand_pos;
    a.e_pair = b->e;
    a.n_pairs = b->n_pairs;
    a.accept = b->accept;
    a.est = b->est;
    a.accept_bits = reinterpret_cast<unsigned long long *>(b->accept_bits);
    a.stream_reads = b->pair_read == nullptr;
    return GK_OK;
}

void drop_graph(gk_ctx *ctx)
{
    if (ctx->graph_exec)
        (void)hipGraphExecDestroy(ctx->graph_exec);
    ctx->graph_exec = nullptr;
    ctx->graph_key.clear();
}

// Scratch for the mixed launch: counters and a residual list able to hold
// every pair of one launch (at most 2^30).
int ensure_mixed_scratch(gk_ctx *ctx, uint64_t n_pairs)
{
    hipError_t e;
    if (!ctx->d_mixed_counters) {
        e = gk_dmalloc(&ctx->d_mixed_counters, 2 * sizeof(uint32_t));
        if (e != hipSuccess)
            return hip_fail(ctx, e, "gk_filter_mixed: hipMalloc counters");
    }
    const uint64_t need = n_pairs < (1ull << 30) ? n_pairs : (1ull << 30);
    if (ctx->resid_cap < need) {
        drop_graph(ctx);
        if (ctx->d_resid)
            (void)hipFree(ctx->d_resid);
        ctx->d_resid = nullptr;
        ctx->resid_cap = 0;
        e = gk_dmalloc(&ctx->d_resid, need * sizeof(uint32_t));
        if (e != hipSuccess)
            return hip_fail(ctx, e, "gk_filter_mixed: hipMalloc residual list");
        ctx->resid_cap = need;
    }
    if (!ctx->capture_stream) {
        e = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking);
        if (e != hipSuccess)
            return hip_fail(ctx, e, "gk_filter_mixed: hipStreamCreate");
    }
    if (!ctx->d_table) {
        e = gk_dmalloc(&ctx->d_table, sizeof(gkd::BatchTable));
        if (e != hipSuccess)
            return hip_fail(ctx, e, "gk_filter_mixed: hipMalloc table");
    }
    for (int k = 0; k < gk_ctx::TABLE_RING; ++k) {
        if (!ctx->h_table[k]) {
            e = gk_hmalloc(&ctx->h_table[k], sizeof(gkd::BatchTable));
            if (e != hipSuccess)
                return hip_fail(ctx, e, "gk_filter_mixed: pinned table");
        }
        if (!ctx->table_ev[k]) {
            e = hipEventCreateWithFlags(&ctx->table_ev[k], hipEventDisableTiming);
            if (e != hipSuccess)
                return hip_fail(ctx, e, "gk_filter_mixed: hipEventCreate");
        }
    }
    return GK_OK;
}

int mixed_args(gk_ctx *ctx, const MixedConfig &c, uint32_t wmax, uint32_t layout,
               gkd::MixedArgs &x)
{
    int per_cu = 0;
    hipError_t e = gkd::mixed_blocks_per_cu(wmax, layout, c.tile, c.ppl, &per_cu);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "gk_filter_mixed: occupancy");
    if (per_cu < 1)
        per_cu = 1;
    const uint32_t bpc = c.blocks_per_cu && (int)c.blocks_per_cu < per_cu ? c.blocks_per_cu
                                                                          : (uint32_t)per_cu;
    x.table = nullptr;
    x.tile_counter = ctx->d_mixed_counters;
    x.resid_count = ctx->d_mixed_counters + 1;
    x.resid_list = ctx->d_resid;
    x.n_tiles = 0;
    x.tile = c.tile;
    x.ppl = c.ppl;
    x.sort_e = c.sort_e;
    x.blocks = bpc * (uint32_t)ctx->cu_count;
    x.resid_blocks = 2u * (uint32_t)ctx->cu_count;
    return GK_OK;
}

}  // namespace

extern "C" {

int gk_filter(gk_ctx *ctx, const gk_batch *b, void *stream)
{
    gkd::TraceRange trace("gk_filter");
    if (!ctx)
        return GK_EINVAL;
    gkd::FilterArgs a{};
    int st = prepare_batch(ctx, b, "gk_filter", a);
    if (st != GK_OK)
        return st == 1 ? GK_OK : st;
    DeviceGuard g(ctx->device);
    if (!g.ok)
        return fail(ctx, GK_EDEVICE, "gk_filter: hipSetDevice failed");
    const uint32_t words = (b->max_read_len + 31) / 32;
    gk_detail_log(ctx, "gk_filter: %llu pairs, %u reads, %u words per mask, layout %u, e %s, "
                  "pairs per lane %u (0: automatic), flags %u",
                  (unsigned long long)b->n_pairs, b->n_reads, words, b->read_layout,
                  b->e ? "per pair" : "uniform", ctx->pairs_per_lane, b->flags);
    hipError_t e = gkd::launch_filter(a, words, b->read_layout, ctx->pairs_per_lane,
                                      (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "gk_filter: launch");
    return GK_OK;
}

int gk_filter_ascii(gk_ctx *ctx, const gk_batch *b, const uint8_t *ascii,
                    const uint64_t *read_off, void *stream)
{
    gkd::TraceRange trace("gk_filter_ascii");
    if (!ctx)
        return GK_EINVAL;
    if (!b)
        return fail(ctx, GK_EINVAL, "gk_filter_ascii: batch is NULL");
    if (b->pair_read)
        return fail(ctx, GK_EINVAL, "gk_filter_ascii: pair_read must be NULL (pair i uses read i)");
    // The batch's read fields are not used: the reads come as text.
    gk_batch bb = *b;
    bb.n_reads = 0;
    bb.pitch = 0;
    bb.reads = nullptr;
    bb.read_len = nullptr;
    bb.read_has_n = nullptr;
    bb.read_layout = GK_READS_SPLIT;
    gkd::FilterArgs a{};
    const int st = prepare_batch(ctx, &bb, "gk_filter_ascii", a);
    if (st != GK_OK)
        return st == 1 ? GK_OK : st;
    if (!ascii || !read_off)
        return fail(ctx, GK_EINVAL, "gk_filter_ascii: NULL ascii or read_off");
    if ((uintptr_t)ascii & 15u)
        return fail(ctx, GK_EINVAL, "gk_filter_ascii: ascii must be 16-byte aligned");
    DeviceGuard g(ctx->device);
    if (!g.ok)
        return fail(ctx, GK_EDEVICE, "gk_filter_ascii: hipSetDevice failed");
    const uint32_t words = (b->max_read_len + 31) / 32;
    gk_detail_log(ctx, "gk_filter_ascii: %llu pairs, %u words per mask, e %s, flags %u",
                  (unsigned long long)b->n_pairs, words, b->e ? "per pair" : "uniform",
                  b->flags);
    const hipError_t e =
        gkd::launch_filter_ascii(a, words, ascii, read_off, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "gk_filter_ascii: launch");
    return GK_OK;
}

int gk_verify(gk_ctx *ctx, const gk_batch *b, const uint8_t *accept, uint16_t *dist,
              void *stream)
{
    gkd::TraceRange trace("gk_verify");
    if (!ctx)
        return GK_EINVAL;
    gkd::FilterArgs a{};
    const int st = prepare_batch(ctx, b, "gk_verify", a);
    if (st == 1)
        return GK_OK;
    if (st != GK_OK)
        return st;
    if (!dist)
        return fail(ctx, GK_EINVAL, "gk_verify: dist is NULL");
    DeviceGuard g(ctx->device);
    if (!g.ok)
        return fail(ctx, GK_EDEVICE, "gk_verify: hipSetDevice failed");
    // The pair list (one word per pair of a chunk of up to 2^30), one word
    // per 4096 of those pairs for the listing's per-workgroup counts, the
    // list of pairs the paired verify kernel leaves to the one-pair kernel,
    // and the key counts and cursors of the listing by length and e.
    const uint64_t need = std::min<uint64_t>(b->n_pairs, 1ull << 30);
    if (need > ctx->verify_cap) {
        if (ctx->d_verify_list)
            (void)hipFree(ctx->d_verify_list);
        ctx->d_verify_list = nullptr;
        ctx->verify_cap = 0;
        hipError_t e = gk_dmalloc(&ctx->d_verify_list,
                                 (2 * need + (need + 4095) / 4096 + gkd::VERIFY_BIN_WORDS) *
                                     sizeof(uint32_t));
        if (e != hipSuccess)
            return hip_fail(ctx, e, "gk_verify: hipMalloc list");
        ctx->verify_cap = need;
    }
    if (!ctx->d_verify_count) {
        hipError_t e = gk_dmalloc(&ctx->d_verify_count, 2 * sizeof(uint32_t));
        if (e != hipSuccess)
            return hip_fail(ctx, e, "gk_verify: hipMalloc count");
    }
    // With a read index per pair and a threshold per pair, the listing orders
    // the pairs by (length, e), which scatters each read's candidates: the
    // one-pair-per-lane kernel then takes the reads from a row-major copy
    // (one run of loads per read instead of a line per transposed row).
    uint32_t *rm = nullptr;
    if (b->pair_read && b->e && b->n_reads > 0) {
        const uint64_t rm_words = (uint64_t)b->n_reads * gkd::verify_rm_stride(a.rows);
        if (rm_words > ctx->reads_rm_cap) {
            if (ctx->d_reads_rm)
                (void)hipFree(ctx->d_reads_rm);
            ctx->d_reads_rm = nullptr;
            ctx->reads_rm_cap = 0;
            hipError_t e = gk_dmalloc(&ctx->d_reads_rm, rm_words * sizeof(uint32_t));
            if (e != hipSuccess)
                return hip_fail(ctx, e, "gk_verify: hipMalloc row-major reads");
            ctx->reads_rm_cap = rm_words;
        }
        rm = ctx->d_reads_rm;
    }
    const uint32_t words = (b->max_read_len + 31) / 32;
    gk_detail_log(ctx, "gk_verify: %llu pairs, %s, pairs listed by %s%s",
                  (unsigned long long)b->n_pairs, accept ? "accepted ones" : "every one",
                  b->e ? "(length, e)" : "length", rm ? ", reads from a row-major copy" : "");
    uint32_t *groups = ctx->d_verify_list + ctx->verify_cap;
    uint32_t *deferred = groups + (ctx->verify_cap + 4095) / 4096;
    uint32_t *bins = deferred + ctx->verify_cap;
    hipError_t e = gkd::launch_verify(a, accept, dist, ctx->d_verify_list, groups, deferred,
                                      ctx->d_verify_count, bins, rm, words, b->read_layout,
                                      ctx->cu_count, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "gk_verify: launch");
    return GK_OK;
}

int gk_filter_mixed(gk_ctx *ctx, const gk_batch *b, void *stream)
{
    gkd::TraceRange trace("gk_filter_mixed");
    if (!ctx)
        return GK_EINVAL;
    gkd::FilterArgs a{};
    int st = prepare_batch(ctx, b, "gk_filter_mixed", a);
    if (st != GK_OK)
        return st == 1 ? GK_OK : st;
    DeviceGuard g(ctx->device);
    if (!g.ok)
        return fail(ctx, GK_EDEVICE, "gk_filter_mixed: hipSetDevice failed");
    if ((st = ensure_mixed_scratch(ctx, b->n_pairs)) != GK_OK)
        return st;
    a.stream_reads = 0;     // the mixed kernel reads each pair entry twice
    const uint32_t wmax = (b->max_read_len + 31) / 32;
    gkd::MixedArgs x{};
    if ((st = mixed_args(ctx, ctx->mixed, wmax, b->read_layout, x)) != GK_OK)
        return st;
    hipError_t e;
    const hipStream_t hs = (hipStream_t)stream;
    // Direct launches: graphs off, variant semantics (their own kernels), or
    // a batch of more than one launch chunk (2^30 pairs).
    if (!ctx->use_graph || a.flags != 0u || b->n_pairs > (1ull << 30)) {
        gk_detail_log(ctx, "gk_filter_mixed: %llu pairs, direct launch (tile %u, %u per lane, "
                      "sort by e %u, %u workgroups)", (unsigned long long)b->n_pairs, x.tile,
                      x.ppl, x.sort_e, x.blocks);
        e = gkd::launch_mixed(a, x, wmax, b->read_layout, hs);
        if (e != hipSuccess)
            return hip_fail(ctx, e, "gk_filter_mixed: launch");
        return GK_OK;
    }
    // Graph: the captured sequence (reset, persistent kernel, residual pass)
    // reads the batch from the context's device table, which a copy on the
    // stream fills before each replay; so one graph serves every batch of a
    // given shape (words per mask, layout) and tuning, captured the first
    // time that pair is seen.
    x.table = ctx->d_table;
    const uint32_t shape[8] = {wmax <= 4 ? 4u : (wmax <= 10 ? 10u : 16u), b->read_layout, x.tile,
                               x.ppl, x.sort_e, x.blocks, x.resid_blocks, 0u};
    std::vector<uint8_t> key(sizeof shape);
    std::memcpy(key.data(), shape, sizeof shape);
    const bool capture = !ctx->graph_exec || key != ctx->graph_key;
    gk_detail_log(ctx, "gk_filter_mixed: %llu pairs, graph %s (words per mask up to %u, tile %u, "
                  "%u per lane, sort by e %u, %u workgroups)", (unsigned long long)b->n_pairs,
                  capture ? "captured" : "replayed", shape[0], x.tile, x.ppl, x.sort_e, x.blocks);
    if (capture) {
        drop_graph(ctx);
        hipGraph_t graph = nullptr;
        e = hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess)
            return hip_fail(ctx, e, "gk_filter_mixed: begin capture");
        hipError_t le = gkd::launch_mixed_table(x, wmax, b->read_layout, ctx->capture_stream);
        e = hipStreamEndCapture(ctx->capture_stream, &graph);
        if (le != hipSuccess || e != hipSuccess) {
            if (graph)
                (void)hipGraphDestroy(graph);
            return hip_fail(ctx, le != hipSuccess ? le : e, "gk_filter_mixed: capture");
        }
        e = hipGraphInstantiate(&ctx->graph_exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            ctx->graph_exec = nullptr;
            return hip_fail(ctx, e, "gk_filter_mixed: instantiate");
        }
        ctx->graph_key = key;
    }
    // This call's table: a pinned slot no earlier replay still reads.
    const int slot = (int)(ctx->table_next++ % gk_ctx::TABLE_RING);
    if (ctx->table_used[slot] && (e = hipEventSynchronize(ctx->table_ev[slot])) != hipSuccess)
        return hip_fail(ctx, e, "gk_filter_mixed: table slot");
    gkd::BatchTable *h = ctx->h_table[slot];
    h->n_batches = 1;
    h->prefix[0] = 0;
    h->prefix[1] = (uint32_t)((b->n_pairs + x.tile - 1) / x.tile);
    h->args[0] = a;
    h->args[0].accept_bits = nullptr;
    const size_t bytes = offsetof(gkd::BatchTable, args) + sizeof(gkd::FilterArgs);
    e = hipMemcpyAsync(ctx->d_table, h, bytes, hipMemcpyHostToDevice, hs);
    if (e == hipSuccess)
        e = hipGraphLaunch(ctx->graph_exec, hs);
    if (e == hipSuccess)
        e = hipEventRecord(ctx->table_ev[slot], hs);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "gk_filter_mixed: graph launch");
    ctx->table_used[slot] = true;
    if (a.accept_bits) {
        e = gkd::launch_accept_bits(a.accept, b->n_pairs, a.accept_bits, hs);
        if (e != hipSuccess)
            return hip_fail(ctx, e, "gk_filter_mixed: accept bits");
    }
    return GK_OK;
}

int gk_filter_mixed_noalloc(gk_ctx *ctx, const gk_batch *b, void *stream)
{
    gkd::TraceRange trace("gk_filter_mixed_noalloc");
    if (!ctx)
        return GK_EINVAL;
    gkd::FilterArgs a{};
    int st = prepare_batch(ctx, b, "gk_filter_mixed_noalloc", a);
    if (st != GK_OK)
        return st == 1 ? GK_OK : st;
    if (b->n_pairs > GK_NOALLOC_MAX_PAIRS)
        return fail(ctx, GK_ERANGE,
                    "gk_filter_mixed_noalloc: n_pairs above GK_NOALLOC_MAX_PAIRS (4194304)");
    uint32_t *scr = scratch_of(ctx->device);
    if (!scr)
        return fail(ctx, GK_EDEVICE, "gk_filter_mixed_noalloc: no scratch address for the device");
    DeviceGuard g(ctx->device);
    if (!g.ok)
        return fail(ctx, GK_EDEVICE, "gk_filter_mixed_noalloc: hipSetDevice failed");
    a.stream_reads = 0;     // the mixed kernel reads each pair entry twice
    const uint32_t wmax = (b->max_read_len + 31) / 32;
    gkd::MixedArgs x{};
    if ((st = mixed_args(ctx, ctx->mixed, wmax, b->read_layout, x)) != GK_OK)
        return st;
    // The same launch sequence as gk_filter_mixed (its first kernel zeroes
    // the two counters), on the library's scratch array and without a graph.
    x.tile_counter = scr;
    x.resid_count = scr + 1;
    x.resid_list = scr + gkd::NOALLOC_LIST_WORD;
    const hipError_t e = gkd::launch_mixed(a, x, wmax, b->read_layout, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "gk_filter_mixed_noalloc: launch");
    return GK_OK;
}

int gk_set_option(gk_ctx *ctx, int option, int64_t value)
{
    if (!ctx)
        return GK_EINVAL;
    switch (option) {
    case GK_OPT_PAIRS_PER_LANE:
        if (value < 0 || value > 65536)
            return fail(ctx, GK_EINVAL, "gk_set_option: pairs per lane must be 0..65536");
        ctx->pairs_per_lane = (uint32_t)value;
        return GK_OK;
    case GK_OPT_MIXED_TILE:
        if (value != 2048 && value != 4096 && value != 8192)
            return fail(ctx, GK_EINVAL, "gk_set_option: mixed tile must be 2048, 4096 or 8192");
        ctx->mixed.tile = (uint32_t)value;
        return GK_OK;
    case GK_OPT_MIXED_PAIRS_PER_LANE:
        if (value != 1 && value != 2)
            return fail(ctx, GK_EINVAL, "gk_set_option: mixed pairs per lane must be 1 or 2");
        ctx->mixed.ppl = (uint32_t)value;
        return GK_OK;
    case GK_OPT_MIXED_SORT_E:
        if (value != 0 && value != 1)
            return fail(ctx, GK_EINVAL, "gk_set_option: mixed sort-by-e must be 0 or 1");
        ctx->mixed.sort_e = (uint32_t)value;
        return GK_OK;
    case GK_OPT_MIXED_BLOCKS_PER_CU:
        if (value < 0 || value > 64)
            return fail(ctx, GK_EINVAL, "gk_set_option: blocks per CU must be 0..64");
        ctx->mixed.blocks_per_cu = (uint32_t)value;
        return GK_OK;
    case GK_OPT_MIXED_GRAPH:
        if (value != 0 && value != 1)
            return fail(ctx, GK_EINVAL, "gk_set_option: graph must be 0 or 1");
        ctx->use_graph = (uint32_t)value;
        return GK_OK;
    case GK_OPT_HOST_ENCODE_THREADS:
        if (value < 0 || value > 64)
            return fail(ctx, GK_EINVAL, "gk_set_option: host encode threads must be 0..64");
        ctx->host_encode_threads = (uint32_t)value;
        return GK_OK;
    case GK_OPT_SERVER_PART_PAIRS:
        if (value < 256 || value > (1ll << 30))
            return fail(ctx, GK_EINVAL, "gk_set_option: server part pairs must be 256..2^30");
        ctx->server_part_pairs = (uint64_t)value;
        return GK_OK;
    case GK_OPT_SERVER_TICK_PAIRS:
        if (value < 4096 || value > (1ll << 26))
            return fail(ctx, GK_EINVAL, "gk_set_option: server tick pairs must be 4096..2^26");
        ctx->server_tick_pairs = (uint64_t)value;
        return GK_OK;
    case GK_OPT_SERVER_COPY_STREAMS:
        if (value < 1 || value > 8)
            return fail(ctx, GK_EINVAL, "gk_set_option: server copy streams must be 1..8");
        ctx->server_copy_streams = (uint32_t)value;
        return GK_OK;
    case GK_OPT_HOST_CHUNK_PAIRS:
        if (value != 0 && (value < 64 || value > (1ll << 26)))
            return fail(ctx, GK_EINVAL, "gk_set_option: host chunk pairs must be 0 or 64..2^26");
        ctx->host_chunk_pairs = (uint64_t)value;
        return GK_OK;
    default:
        return fail(ctx, GK_EINVAL, "gk_set_option: unknown option");
    }
}

int gk_get_option(const gk_ctx *ctx, int option, int64_t *value)
{
    if (!ctx || !value)
        return GK_EINVAL;
    switch (option) {
    case GK_OPT_PAIRS_PER_LANE:
        *value = ctx->pairs_per_lane;
        return GK_OK;
    case GK_OPT_MIXED_TILE:
        *value = ctx->mixed.tile;
        return GK_OK;
    case GK_OPT_MIXED_PAIRS_PER_LANE:
        *value = ctx->mixed.ppl;
        return GK_OK;
    case GK_OPT_MIXED_SORT_E:
        *value = ctx->mixed.sort_e;
        return GK_OK;
    case GK_OPT_MIXED_BLOCKS_PER_CU:
        *value = ctx->mixed.blocks_per_cu;
        return GK_OK;
    case GK_OPT_MIXED_GRAPH:
        *value = ctx->use_graph;
        return GK_OK;
    case GK_OPT_HOST_ENCODE_THREADS:
        *value = ctx->host_encode_threads;
        return GK_OK;
    case GK_OPT_SERVER_PART_PAIRS:
        *value = (int64_t)ctx->server_part_pairs;
        return GK_OK;
    case GK_OPT_SERVER_TICK_PAIRS:
        *value = (int64_t)ctx->server_tick_pairs;
        return GK_OK;
    case GK_OPT_HOST_CHUNK_PAIRS:
        *value = (int64_t)ctx->host_chunk_pairs;
        return GK_OK;
    case GK_OPT_SERVER_COPY_STREAMS:
        *value = ctx->server_copy_streams;
        return GK_OK;
    default:
        return GK_EINVAL;
    }
}

int gk_tune_mixed(gk_ctx *ctx, const gk_batch *b, void *stream, uint64_t sample_pairs,
                  const char *cache_path, char *report, size_t report_cap)
{
    gkd::TraceRange trace("gk_tune_mixed");
    if (!ctx)
        return GK_EINVAL;
    gkd::FilterArgs a{};
    int st = prepare_batch(ctx, b, "gk_tune_mixed", a);
    if (st != GK_OK)
        return st == 1 ? GK_OK : st;
    DeviceGuard g(ctx->device);
    if (!g.ok)
        return fail(ctx, GK_EDEVICE, "gk_tune_mixed: hipSetDevice failed");
    if ((st = ensure_mixed_scratch(ctx, b->n_pairs)) != GK_OK)
        return st;
    a.stream_reads = 0;
    const uint32_t wmax = (b->max_read_len + 31) / 32;
    const uint64_t n_full = b->n_pairs;
    if (sample_pairs && sample_pairs < a.n_pairs)
        a.n_pairs = sample_pairs;
    a.accept_bits = nullptr;

    // Key: device, CU count, words per mask, layout, threshold mode, batch
    // size (power-of-two bucket).
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, ctx->device) != hipSuccess)
        return fail(ctx, GK_EDEVICE, "gk_tune_mixed: device properties");
    std::ostringstream k;
    k << prop.gcnArchName << "|cu=" << ctx->cu_count << "|w=" << wmax
      << "|layout=" << b->read_layout << "|e="
      << (b->e ? std::string("per-pair") : "uniform:" + std::to_string(b->e_uniform))
      << "|n=2^" << (int)std::floor(std::log2((double)n_full));
    const std::string key = k.str();
    std::ostringstream rep;

    auto parse = [](const std::string &line, const char *field, long &out) {
        const std::string f = std::string("\"") + field + "\": ";
        const size_t p = line.find(f);
        if (p == std::string::npos)
            return false;
        out = std::strtol(line.c_str() + p + f.size(), nullptr, 10);
        return true;
    };
    auto give = [&](const char *source, const MixedConfig &c) {
        rep << "{\"key\": \"" << key << "\", \"source\": \"" << source << "\", \"tile\": "
            << c.tile << ", \"ppl\": " << c.ppl << ", \"sort_e\": " << c.sort_e
            << ", \"blocks_per_cu\": " << c.blocks_per_cu << "}";
        if (report && report_cap) {
            std::strncpy(report, rep.str().c_str(), report_cap - 1);
            report[report_cap - 1] = 0;
        }
        gk_detail_log(ctx, "gk_tune_mixed: %s, %s: tile %u, %u per lane, sort by e %u, "
                      "%u workgroups per CU (0: full)", key.c_str(), source, c.tile, c.ppl,
                      c.sort_e, c.blocks_per_cu);
        return GK_OK;
    };
    if (ctx->autotune == AUTOTUNE_OFF)
        return give("off", ctx->mixed);
    if (cache_path && *cache_path && ctx->autotune == AUTOTUNE_USE) {
        // The last valid line for the key: a refresh appends after older ones.
        std::ifstream in(cache_path);
        std::string line;
        const std::string needle = "\"key\": \"" + key + "\"";
        bool found = false;
        MixedConfig cached;
        while (std::getline(in, line)) {
            if (line.find(needle) == std::string::npos)
                continue;
            long t, p, se, bpc;
            if (parse(line, "tile", t) && parse(line, "ppl", p) && parse(line, "sort_e", se) &&
                parse(line, "blocks_per_cu", bpc) && (t == 2048 || t == 4096 || t == 8192) &&
                (p == 1 || p == 2) && (se == 0 || se == 1) && bpc >= 0 && bpc <= 64) {
                cached = MixedConfig{(uint32_t)t, (uint32_t)p, (uint32_t)se, (uint32_t)bpc};
                found = true;
            }
        }
        if (found) {
            ctx->mixed = cached;
            drop_graph(ctx);
            return give("cache", cached);
        }
    }

    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(ctx, GK_EDEVICE, "gk_tune_mixed: hipEventCreate");
    const hipStream_t s = (hipStream_t)stream;
    int full_bpc = 0;
    MixedConfig best;
    float best_ms = -1.f;
    rep << "{\"key\": \"" << key << "\", \"source\": \"measured\", \"sample_pairs\": " << a.n_pairs
        << ", \"candidates\": [";
    bool first = true;
    hipError_t err = hipSuccess;
    for (uint32_t tile : {2048u, 4096u, 8192u}) {
        for (uint32_t ppl : {1u, 2u}) {
            if (ppl == 2 && wmax > 10)
                continue;                      // two pairs per lane only up to 10 words
            if ((err = gkd::mixed_blocks_per_cu(wmax, b->read_layout, tile, ppl, &full_bpc)) !=
                hipSuccess)
                break;
            for (uint32_t sort_e : {0u, 1u})
                for (uint32_t bpc : {0u, (uint32_t)std::max(1, full_bpc / 2)}) {
                    MixedConfig c{tile, ppl, sort_e, bpc};
                    gkd::MixedArgs x{};
                    if ((st = mixed_args(ctx, c, wmax, b->read_layout, x)) != GK_OK) {
                        (void)hipEventDestroy(e0);
                        (void)hipEventDestroy(e1);
                        return st;
                    }
                    float times[5];
                    for (int rep_i = -1; rep_i < 5 && err == hipSuccess; ++rep_i) {
                        err = hipEventRecord(e0, s);
                        if (err == hipSuccess)
                            err = gkd::launch_mixed(a, x, wmax, b->read_layout, s);
                        if (err == hipSuccess)
                            err = hipEventRecord(e1, s);
                        if (err == hipSuccess)
                            err = hipEventSynchronize(e1);
                        float ms = 0;
                        if (err == hipSuccess)
                            err = hipEventElapsedTime(&ms, e0, e1);
                        if (rep_i >= 0)
                            times[rep_i] = ms;
                    }
                    if (err != hipSuccess)
                        break;
                    std::sort(times, times + 5);
                    const float med = times[2];
                    rep << (first ? "" : ", ") << "{\"tile\": " << tile << ", \"ppl\": " << ppl
                        << ", \"sort_e\": " << sort_e << ", \"blocks_per_cu\": " << bpc
                        << ", \"ms\": " << med << "}";
                    first = false;
                    if (best_ms < 0 || med < best_ms) {
                        best_ms = med;
                        best = c;
                    }
                }
            if (err != hipSuccess)
                break;
        }
        if (err != hipSuccess)
            break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess)
        return hip_fail(ctx, err, "gk_tune_mixed: timing");
    ctx->mixed = best;
    drop_graph(ctx);
    rep << "], \"tile\": " << best.tile << ", \"ppl\": " << best.ppl << ", \"sort_e\": "
        << best.sort_e << ", \"blocks_per_cu\": " << best.blocks_per_cu << ", \"ms\": " << best_ms
        << "}";
    if (cache_path && *cache_path) {
        std::ofstream out(cache_path, std::ios::app);
        out << "{\"key\": \"" << key << "\", \"tile\": " << best.tile << ", \"ppl\": " << best.ppl
            << ", \"sort_e\": " << best.sort_e << ", \"blocks_per_cu\": " << best.blocks_per_cu
            << ", \"ms\": " << best_ms << "}\n";
    }
    if (report && report_cap) {
        std::strncpy(report, rep.str().c_str(), report_cap - 1);
        report[report_cap - 1] = 0;
    }
    gk_detail_log(ctx, "gk_tune_mixed: %s, measured: tile %u, %u per lane, sort by e %u, "
                  "%u workgroups per CU (0: full), %.4f ms", key.c_str(), best.tile, best.ppl,
                  best.sort_e, best.blocks_per_cu, best_ms);
    return GK_OK;
}

}  // extern "C"

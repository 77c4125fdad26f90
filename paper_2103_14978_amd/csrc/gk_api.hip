// Host side of libgk: context, resident reference, argument checks, launches.
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "gk_internal.h"

namespace {

thread_local std::string g_create_error;

// Makes the context's device current for the duration of a call and restores
// the caller's device afterwards.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess)
            prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0)
            (void)hipSetDevice(prev);
    }
};

int fail(gk_ctx *ctx, int code, const std::string &msg)
{
    if (ctx)
        ctx->err = msg;
    return code;
}

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
    ctx->ref_planes = nullptr;
    ctx->ref_unk = nullptr;
    ctx->ref_len = ctx->ref_words = ctx->ref_unknown = 0;
}

}  // namespace

extern "C" {

int gk_create(int device, gk_ctx **out)
{
    if (!out) {
        g_create_error = "gk_create: out is NULL";
        return GK_EINVAL;
    }
    *out = nullptr;
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
    e = hipMalloc(&ctx->d_counter, sizeof(unsigned long long));
    if (e != hipSuccess) {
        delete ctx;
        g_create_error = std::string("gk_create: hipMalloc: ") + hipGetErrorName(e);
        return e == hipErrorOutOfMemory ? GK_ENOMEM : GK_EDEVICE;
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
    }
    delete ctx;
}

const char *gk_last_error(const gk_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

int gk_load_reference(gk_ctx *ctx, const char *ascii, uint64_t len)
{
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
    hipError_t e = hipMalloc(&ctx->ref_planes, alloc_words * sizeof(uint2));
    if (e != hipSuccess)
        return free_reference(ctx), hip_fail(ctx, e, "gk_load_reference: hipMalloc planes");
    e = hipMalloc(&ctx->ref_unk, alloc_words * sizeof(uint32_t));
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
    e = hipMalloc(&stage, step);
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
    if (e != hipSuccess)
        return free_reference(ctx), hip_fail(ctx, e, "gk_load_reference: pack");
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
                    uint32_t pitch, uint32_t rows, uint32_t *packed_out, uint16_t *len_out,
                    uint8_t *has_n_out, void *stream)
{
    if (!ctx)
        return GK_EINVAL;
    if (n_reads == 0)
        return GK_OK;
    if (!ascii || !read_off || !packed_out || !len_out)
        return fail(ctx, GK_EINVAL, "gk_encode_reads: NULL buffer");
    if (pitch < n_reads)
        return fail(ctx, GK_EINVAL, "gk_encode_reads: pitch < n_reads");
    if (rows < 1 || rows > 32)
        return fail(ctx, GK_EINVAL, "gk_encode_reads: rows must be 1..32");
    DeviceGuard g(ctx->device);
    if (!g.ok)
        return fail(ctx, GK_EDEVICE, "gk_encode_reads: hipSetDevice failed");
    hipError_t e = gkd::launch_encode_reads(ascii, read_off, n_reads, pitch, rows, packed_out,
                                            len_out, has_n_out, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "gk_encode_reads: launch");
    return GK_OK;
}

int gk_filter(gk_ctx *ctx, const gk_batch *b, void *stream)
{
    if (!ctx)
        return GK_EINVAL;
    if (!b)
        return fail(ctx, GK_EINVAL, "gk_filter: batch is NULL");
    if (!ctx->ref_planes)
        return fail(ctx, GK_ENOREF, "gk_filter: no reference loaded");
    if (b->max_read_len < 1 || b->max_read_len > GK_MAX_READ_LEN)
        return fail(ctx, GK_EINVAL, "gk_filter: max_read_len must be 1..512");
    if (b->e_uniform > 255)
        return fail(ctx, GK_EINVAL, "gk_filter: e_uniform must be 0..255");
    if (b->pitch < b->n_reads)
        return fail(ctx, GK_EINVAL, "gk_filter: pitch < n_reads");
    if (b->n_pairs == 0)
        return GK_OK;
    if (b->n_pairs >= (1ull << 38))
        return fail(ctx, GK_ERANGE, "gk_filter: n_pairs must be below 2^38");
    if (!b->pair_read || !b->cand_pos || !b->accept || !b->est)
        return fail(ctx, GK_EINVAL, "gk_filter: NULL pair or output buffer");
    if (b->n_reads > 0 && (!b->reads || !b->read_len))
        return fail(ctx, GK_EINVAL, "gk_filter: NULL read buffer");
    DeviceGuard g(ctx->device);
    if (!g.ok)
        return fail(ctx, GK_EDEVICE, "gk_filter: hipSetDevice failed");

    gkd::FilterArgs a;
    a.ref_planes = ctx->ref_planes;
    a.ref_unk = ctx->ref_unk;
    a.ref_len = ctx->ref_len;
    a.ref_has_unknown = ctx->ref_unknown > 0;
    a.n_reads = b->n_reads;
    a.pitch = b->pitch;
    a.e_uniform = b->e_uniform;
    a.max_read_len = b->max_read_len;
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
    const uint32_t words = (b->max_read_len + 31) / 32;
    hipError_t e = gkd::launch_filter(a, words, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "gk_filter: launch");
    return GK_OK;
}

}  // extern "C"

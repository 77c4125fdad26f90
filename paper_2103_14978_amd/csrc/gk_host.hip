// Host-to-host filter (gk_filter_host): reads and pairs in host memory,
// results back in host memory, as the paper's filter time counts them
// (Sec. 4.3).  The batch is cut into chunks; for each chunk the copies in,
// the read encoding (Sec. 3.3), the filter and the copies out run on three
// streams, so chunk j's copies overlap chunk j-1's kernels and chunk j-2's
// copies out.  The paper instead preprocesses a whole batch, then filters it,
// then copies it back (Sec. 3.5).
#include <algorithm>
#include <string>
#include <vector>

#include "gk_internal.h"

namespace {

int fail(gk_ctx *ctx, int code, const std::string &msg) { return gk_detail_fail(ctx, code, msg); }

int hip_fail(gk_ctx *ctx, hipError_t e, const char *what)
{
    std::string msg = std::string("gk_filter_host: ") + what + ": " + hipGetErrorName(e) + " (" +
                      hipGetErrorString(e) + ")";
    return fail(ctx, e == hipErrorOutOfMemory ? GK_ENOMEM : GK_EDEVICE, msg);
}

template <typename T>
void release(T *&p)
{
    if (p)
        (void)hipFree(p);
    p = nullptr;
}

template <typename T>
hipError_t realloc_device(T *&p, uint64_t count)
{
    release(p);
    return gk_dmalloc(&p, std::max<uint64_t>(count, 1) * sizeof(T));
}

// Grows the buffers to the batch (never shrinks them).
hipError_t ensure_buffers(HostPipe &h, uint64_t ascii_bytes, uint64_t n_reads,
                          uint64_t packed_words, uint64_t n_pairs, uint32_t chunks)
{
    hipError_t e = hipSuccess;
    if (!h.s_in) {
        e = hipStreamCreateWithFlags(&h.s_in, hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipStreamCreateWithFlags(&h.s_comp, hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipStreamCreateWithFlags(&h.s_out, hipStreamNonBlocking);
        if (e != hipSuccess)
            return e;
    }
    while (h.ev_in.size() < chunks) {
        hipEvent_t a = nullptr, b = nullptr;
        e = hipEventCreateWithFlags(&a, hipEventDisableTiming);
        if (e != hipSuccess)
            return e;
        e = hipEventCreateWithFlags(&b, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipEventDestroy(a);
            return e;
        }
        h.ev_in.push_back(a);
        h.ev_comp.push_back(b);
    }
    // Up to 4 bytes past the last read byte may be touched by aligned loads.
    if (ascii_bytes + 64 > h.ascii_cap) {
        h.ascii_cap = 0;
        if ((e = realloc_device(h.ascii, ascii_bytes + 64)) != hipSuccess)
            return e;
        h.ascii_cap = ascii_bytes + 64;
    }
    if (n_reads > h.read_cap || h.off == nullptr) {
        h.read_cap = 0;
        if ((e = realloc_device(h.off, n_reads + 1)) != hipSuccess ||
            (e = realloc_device(h.len, n_reads)) != hipSuccess ||
            (e = realloc_device(h.has_n, n_reads)) != hipSuccess)
            return e;
        h.read_cap = n_reads;
    }
    if (packed_words > h.packed_cap || h.packed == nullptr) {
        h.packed_cap = 0;
        if ((e = realloc_device(h.packed, packed_words)) != hipSuccess)
            return e;
        h.packed_cap = packed_words;
    }
    if (n_pairs > h.pair_cap || h.cand_pos == nullptr) {
        h.pair_cap = 0;
        if ((e = realloc_device(h.pair_read, n_pairs)) != hipSuccess ||
            (e = realloc_device(h.cand_pos, n_pairs)) != hipSuccess ||
            (e = realloc_device(h.e, n_pairs)) != hipSuccess ||
            (e = realloc_device(h.accept, n_pairs)) != hipSuccess ||
            (e = realloc_device(h.est, n_pairs)) != hipSuccess)
            return e;
        h.pair_cap = n_pairs;
    }
    return hipSuccess;
}

}  // namespace

void gk_detail_free_host_pipe(gk_ctx *ctx)
{
    HostPipe &h = ctx->host;
    release(h.ascii);
    release(h.off);
    release(h.packed);
    release(h.len);
    release(h.has_n);
    release(h.pair_read);
    release(h.cand_pos);
    release(h.e);
    release(h.accept);
    release(h.est);
    h.ascii_cap = h.read_cap = h.packed_cap = h.pair_cap = 0;
    for (hipEvent_t ev : h.ev_in)
        (void)hipEventDestroy(ev);
    for (hipEvent_t ev : h.ev_comp)
        (void)hipEventDestroy(ev);
    h.ev_in.clear();
    h.ev_comp.clear();
    for (uint8_t *&st : h.stage) {
        if (st)
            (void)hipHostFree(st);
        st = nullptr;
    }
    h.stage_cap = 0;
    h.pool.reset();
    h.pool_threads = 0;
    for (hipStream_t *s : {&h.s_in, &h.s_comp, &h.s_out}) {
        if (*s)
            (void)hipStreamDestroy(*s);
        *s = nullptr;
    }
}

extern "C" int gk_filter_host(gk_ctx *ctx, const gk_host_batch *b)
{
    if (!ctx)
        return GK_EINVAL;
    if (!b)
        return fail(ctx, GK_EINVAL, "gk_filter_host: batch is NULL");
    if (!ctx->ref_planes)
        return fail(ctx, GK_ENOREF, "gk_filter_host: no reference loaded");
    if (b->max_read_len < 1 || b->max_read_len > GK_MAX_READ_LEN)
        return fail(ctx, GK_EINVAL, "gk_filter_host: max_read_len must be 1..512");
    if (b->e_uniform > 255)
        return fail(ctx, GK_EINVAL, "gk_filter_host: e_uniform must be 0..255");
    if (b->n_reads >= (1u << 30))
        return fail(ctx, GK_EINVAL, "gk_filter_host: n_reads must be below 2^30");
    if (b->flags & ~(GK_FLAG_NO_REFINE | GK_FLAG_HAMMING_FASTPATH))
        return fail(ctx, GK_EINVAL, "gk_filter_host: unknown flags");
    if (b->n_pairs == 0)
        return GK_OK;
    if (b->n_pairs >= (1ull << 38))
        return fail(ctx, GK_ERANGE, "gk_filter_host: n_pairs must be below 2^38");
    if (!b->cand_pos || !b->accept || !b->est)
        return fail(ctx, GK_EINVAL, "gk_filter_host: NULL pair or output buffer");
    if (!b->pair_read && b->n_pairs != b->n_reads)
        return fail(ctx, GK_EINVAL, "gk_filter_host: pair_read NULL needs n_pairs == n_reads");
    const bool host_encoded = b->packed != nullptr;
    if (host_encoded) {
        if (b->n_reads > 0 && !b->read_len)
            return fail(ctx, GK_EINVAL, "gk_filter_host: packed reads need read_len");
        if (b->packed_layout != GK_READS_SPLIT && b->packed_layout != GK_READS_INTERLEAVED)
            return fail(ctx, GK_EINVAL, "gk_filter_host: unknown packed_layout");
    } else {
        if (b->n_reads > 0 && (!b->ascii || !b->read_off))
            return fail(ctx, GK_EINVAL, "gk_filter_host: NULL read buffer");
        if (b->n_reads > 0 && b->read_off[0] != 0)
            return fail(ctx, GK_EINVAL, "gk_filter_host: read_off[0] must be 0");
    }
    DeviceScope g(ctx->device);
    if (!g.ok)
        return fail(ctx, GK_EDEVICE, "gk_filter_host: hipSetDevice failed");

    const uint64_t nr = b->n_reads, np = b->n_pairs;
    const uint32_t pitch = (uint32_t)std::max<uint64_t>(64, (nr + 63) / 64 * 64);
    const uint32_t rows = (b->max_read_len + 15) / 16;
    // ASCII reads encoded here on host threads (GK_OPT_HOST_ENCODE_THREADS):
    // 2-bit rows cross the bus, as for reads the caller encoded.
    const bool encode_here = !host_encoded && ctx->host_encode_threads > 0 && nr > 0;
    const bool rows_in = host_encoded || encode_here;
    const uint64_t text_bytes = (!host_encoded && nr) ? b->read_off[nr] : 0;
    // ASCII text, or 2-bit rows staged in the same buffer.
    const uint64_t bytes = rows_in ? nr * rows * sizeof(uint32_t) : text_bytes;
    const bool identity = b->pair_read == nullptr;

    // Chunks of at least 2^20 pairs, at most 16 of them.
    const uint32_t K = (uint32_t)std::min<uint64_t>(16, std::max<uint64_t>(1, (np + (1u << 20) - 1) >> 20));
    const uint64_t P = ((np + K - 1) / K + 63) / 64 * 64;           // pairs per chunk
    const uint64_t R = identity ? P : std::max<uint64_t>(1, (nr + K - 1) / K);  // reads per chunk

    HostPipe &h = ctx->host;
    hipError_t e = ensure_buffers(h, bytes, nr, (uint64_t)rows * pitch, np, K);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "device buffers");
    // Two pinned staging buffers, each one read chunk of rows, lengths and
    // unknown-base flags; chunk j uses buffer j % 2 once chunk j - 2's copy
    // from it is done.
    const uint64_t stage_rows_bytes = R * rows * sizeof(uint32_t);
    const uint64_t stage_bytes = stage_rows_bytes + R * sizeof(uint16_t) + R;
    if (encode_here) {
        if (stage_bytes > h.stage_cap) {
            for (uint8_t *&st : h.stage) {
                if (st)
                    (void)hipHostFree(st);
                st = nullptr;
            }
            h.stage_cap = 0;
            for (uint8_t *&st : h.stage)
                if ((e = gk_hmalloc((void **)&st, stage_bytes)) !=
                    hipSuccess)
                    return hip_fail(ctx, e, "pinned staging");
            h.stage_cap = stage_bytes;
        }
        if (h.pool_threads != ctx->host_encode_threads) {
            h.pool.reset();
            h.pool.reset(new gkd::HostEncodePool(ctx->host_encode_threads));
            h.pool_threads = ctx->host_encode_threads;
        }
    }

    std::vector<uint32_t> need(K, 0);   // last read chunk each pair chunk needs
    bool bad_offsets = false;
    uint32_t next_q = 0;
    for (uint32_t j = 0; j < K && e == hipSuccess; ++j) {
        // Read chunk j: offsets must be non-decreasing and within the text.
        const uint64_t r0 = std::min<uint64_t>(nr, (uint64_t)j * R);
        const uint64_t r1 = std::min<uint64_t>(nr, r0 + R);
        uint32_t *rows_dev =
            rows_in ? reinterpret_cast<uint32_t *>(h.ascii) + r0 * rows : nullptr;
        if (r1 > r0 && encode_here) {
            for (uint64_t r = r0; r < r1 && !bad_offsets; ++r)
                bad_offsets = b->read_off[r + 1] < b->read_off[r];
            bad_offsets = bad_offsets || b->read_off[r1] > text_bytes;
            if (bad_offsets)
                break;
            if (j >= 2)
                e = hipEventSynchronize(h.ev_in[j - 2]);
            uint8_t *st = h.stage[j & 1u];
            uint32_t *rows_h = reinterpret_cast<uint32_t *>(st);
            uint16_t *len_h = reinterpret_cast<uint16_t *>(st + stage_rows_bytes);
            uint8_t *has_n_h = st + stage_rows_bytes + R * sizeof(uint16_t);
            if (e == hipSuccess) {
                const uint64_t cnt = r1 - r0;
                h.pool->run([&](unsigned i, unsigned n) {
                    const uint64_t a = r0 + cnt * i / n, z = r0 + cnt * (i + 1) / n;
                    gkd::host_encode_rows(b->ascii, text_bytes, b->read_off, a, z, rows,
                                          rows_h + (a - r0) * rows, len_h + (a - r0),
                                          has_n_h + (a - r0));
                });
                e = hipMemcpyAsync(rows_dev, rows_h, cnt * rows * sizeof(uint32_t),
                                   hipMemcpyHostToDevice, h.s_in);
            }
            if (e == hipSuccess)
                e = hipMemcpyAsync(h.len + r0, len_h, (r1 - r0) * sizeof(uint16_t),
                                   hipMemcpyHostToDevice, h.s_in);
            if (e == hipSuccess)
                e = hipMemcpyAsync(h.has_n + r0, has_n_h, r1 - r0, hipMemcpyHostToDevice,
                                   h.s_in);
        } else if (r1 > r0 && host_encoded) {
            e = hipMemcpyAsync(rows_dev, b->packed + r0 * rows,
                               (r1 - r0) * rows * sizeof(uint32_t), hipMemcpyHostToDevice,
                               h.s_in);
            if (e == hipSuccess)
                e = hipMemcpyAsync(h.len + r0, b->read_len + r0, (r1 - r0) * sizeof(uint16_t),
                                   hipMemcpyHostToDevice, h.s_in);
            if (e == hipSuccess)
                e = b->read_has_n
                        ? hipMemcpyAsync(h.has_n + r0, b->read_has_n + r0, r1 - r0,
                                         hipMemcpyHostToDevice, h.s_in)
                        : hipMemsetAsync(h.has_n + r0, 0, r1 - r0, h.s_in);
        } else if (r1 > r0) {
            for (uint64_t r = r0; r < r1 && !bad_offsets; ++r)
                bad_offsets = b->read_off[r + 1] < b->read_off[r];
            bad_offsets = bad_offsets || b->read_off[r1] > bytes;
            if (bad_offsets)
                break;
            const uint64_t a0 = b->read_off[r0], a1 = b->read_off[r1];
            if (a1 > a0)
                e = hipMemcpyAsync(h.ascii + a0, b->ascii + a0, a1 - a0, hipMemcpyHostToDevice,
                                   h.s_in);
            if (e == hipSuccess)
                e = hipMemcpyAsync(h.off + r0, b->read_off + r0, (r1 - r0 + 1) * sizeof(uint64_t),
                                   hipMemcpyHostToDevice, h.s_in);
        }
        // Pair chunk j.
        const uint64_t p0 = std::min<uint64_t>(np, (uint64_t)j * P);
        const uint64_t p1 = std::min<uint64_t>(np, p0 + P);
        if (e == hipSuccess && p1 > p0) {
            e = hipMemcpyAsync(h.cand_pos + p0, b->cand_pos + p0, (p1 - p0) * sizeof(uint32_t),
                               hipMemcpyHostToDevice, h.s_in);
            if (e == hipSuccess && b->e)
                e = hipMemcpyAsync(h.e + p0, b->e + p0, p1 - p0, hipMemcpyHostToDevice, h.s_in);
            if (e == hipSuccess && !identity)
                e = hipMemcpyAsync(h.pair_read + p0, b->pair_read + p0,
                                   (p1 - p0) * sizeof(uint32_t), hipMemcpyHostToDevice, h.s_in);
        }
        if (!identity && p1 > p0 && nr > 0) {
            uint32_t mx = 0;
            for (uint64_t i = p0; i < p1; ++i) {
                const uint32_t r = b->pair_read[i];
                if (r < nr && r > mx)
                    mx = r;          // pairs of reads >= n_reads are GK_INVALID
            }
            need[j] = (uint32_t)std::min<uint64_t>(K - 1, mx / R);
        } else {
            need[j] = j;
        }
        if (e == hipSuccess)
            e = hipEventRecord(h.ev_in[j], h.s_in);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(h.s_comp, h.ev_in[j], 0);
        if (e == hipSuccess && r1 > r0)
            e = rows_in
                    ? gkd::launch_transpose_reads(rows_dev, (uint32_t)(r1 - r0), rows, pitch,
                                                  h.packed + r0, h.s_comp)
                    : gkd::launch_encode_reads(h.ascii, h.off + r0, (uint32_t)(r1 - r0), pitch,
                                               rows, GK_READS_SPLIT, h.packed + r0, h.len + r0,
                                               h.has_n + r0, h.s_comp);
        // Filter every pair chunk whose reads are now encoded, in order.
        while (e == hipSuccess && next_q <= j && need[next_q] <= j) {
            const uint32_t q = next_q++;
            const uint64_t q0 = std::min<uint64_t>(np, (uint64_t)q * P);
            const uint64_t q1 = std::min<uint64_t>(np, q0 + P);
            if (q1 == q0)
                continue;
            gk_batch fb{};
            fb.pitch = pitch;
            fb.max_read_len = b->max_read_len;
            fb.e_uniform = b->e_uniform;
            fb.read_layout = host_encoded ? b->packed_layout : GK_READS_SPLIT;   // encode_here: split
            fb.flags = b->flags;
            fb.n_pairs = q1 - q0;
            fb.cand_pos = h.cand_pos + q0;
            fb.e = b->e ? h.e + q0 : nullptr;
            fb.accept = h.accept + q0;
            fb.est = h.est + q0;
            if (identity) {            // pair i of the chunk uses read q0 + i
                fb.n_reads = (uint32_t)(q1 - q0);
                fb.reads = h.packed + q0;
                fb.read_len = h.len + q0;
                fb.read_has_n = h.has_n + q0;
                fb.pair_read = nullptr;
            } else {
                fb.n_reads = (uint32_t)nr;
                fb.reads = h.packed;
                fb.read_len = h.len;
                fb.read_has_n = h.has_n;
                fb.pair_read = h.pair_read + q0;
            }
            const int st = gk_filter(ctx, &fb, h.s_comp);
            if (st != GK_OK) {
                (void)hipStreamSynchronize(h.s_in);
                (void)hipStreamSynchronize(h.s_comp);
                (void)hipStreamSynchronize(h.s_out);
                return st;
            }
            e = hipEventRecord(h.ev_comp[q], h.s_comp);
            if (e == hipSuccess)
                e = hipStreamWaitEvent(h.s_out, h.ev_comp[q], 0);
            if (e == hipSuccess)
                e = hipMemcpyAsync(b->accept + q0, h.accept + q0, q1 - q0, hipMemcpyDeviceToHost,
                                   h.s_out);
            if (e == hipSuccess)
                e = hipMemcpyAsync(b->est + q0, h.est + q0, (q1 - q0) * sizeof(uint16_t),
                                   hipMemcpyDeviceToHost, h.s_out);
        }
    }
    const hipError_t e1 = hipStreamSynchronize(h.s_in);
    const hipError_t e2 = hipStreamSynchronize(h.s_comp);
    const hipError_t e3 = hipStreamSynchronize(h.s_out);
    if (e == hipSuccess)
        e = e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : e3);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "pipeline");
    if (bad_offsets)
        return fail(ctx, GK_EINVAL, "gk_filter_host: read_off decreases or passes the text end");
    ctx->err.clear();
    return GK_OK;
}

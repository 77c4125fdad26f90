// Host-to-host filter (gk_filter_host): reads and pairs in host memory,
// results back in host memory, as the paper's filter time counts them
// (Sec. 4.3).  The batch is cut into chunks; for each chunk the copies in,
// the read encoding (Sec. 3.3), the filter and the copies out run on three
// streams, so chunk j's copies overlap chunk j-1's kernels and chunk j-2's
// copies out.  The chunks cycle through a ring of three device slots, so the
// device memory is set by the chunk size, not by the batch.  The paper
// instead preprocesses a whole batch, then filters it, then copies it back
// (Sec. 3.5).
#include <algorithm>
#include <string>
#include <cstdint>

#include "gk_internal.h"
#include "gk_trace.h"

namespace {

int fail(gk_ctx *ctx, int code, const std::string &msg) { return gk_detail_fail(ctx, code, msg); }

int hip_fail(gk_ctx *ctx, hipError_t e, const char *what)
{
    std::string msg = std::string("gk_filter_host: ") + what + ": " + hipGetErrorName(e) + " (" +
                      hipGetErrorString(e) + ")";
    return fail(ctx, e == hipErrorOutOfMemory ? GK_ENOMEM : GK_EDEVICE, msg);
}

template <typename T>
void release(DevBuf<T> &b)
{
    if (b.p)
        (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

// Grows b to at least n elements (never shrinks it).
template <typename T>
hipError_t fit(DevBuf<T> &b, uint64_t n)
{
    n = std::max<uint64_t>(n, 1);
    if (b.p && b.cap >= n)
        return hipSuccess;
    release(b);
    const hipError_t e = gk_dmalloc(&b.p, n * sizeof(T));
    if (e == hipSuccess)
        b.cap = n;
    return e;
}

void release(HostReads &r)
{
    release(r.text);
    release(r.off);
    release(r.len);
    release(r.has_n);
    release(r.packed);
}

// Room for n_reads reads of text_bytes bytes of text (or row-major words)
// and packed_words transposed words.
hipError_t fit(HostReads &r, uint64_t text_bytes, uint64_t n_reads, uint64_t packed_words)
{
    hipError_t e = fit(r.text, text_bytes);
    if (e == hipSuccess)
        e = fit(r.off, n_reads + 1);
    if (e == hipSuccess)
        e = fit(r.len, n_reads);
    if (e == hipSuccess)
        e = fit(r.has_n, n_reads);
    if (e == hipSuccess)
        e = fit(r.packed, packed_words);
    return e;
}

hipError_t make_event(hipEvent_t &ev)
{
    return ev ? hipSuccess : hipEventCreateWithFlags(&ev, hipEventDisableTiming);
}

hipError_t ensure_streams(HostPipe &h)
{
    hipError_t e = hipSuccess;
    for (hipStream_t *s : {&h.s_in, &h.s_comp, &h.s_out})
        if (e == hipSuccess && !*s)
            e = hipStreamCreateWithFlags(s, hipStreamNonBlocking);
    for (HostSlot &sl : h.slot)
        for (hipEvent_t *ev : {&sl.ev_in, &sl.ev_comp, &sl.ev_out})
            if (e == hipSuccess)
                e = make_event(*ev);
    for (hipEvent_t &ev : h.ev_read)
        if (e == hipSuccess)
            e = make_event(ev);
    return e;
}

// Pairs per chunk: the option, else n_pairs / 16 within [2^20, 2^22]; never
// more than the batch; a multiple of 64.
uint64_t chunk_pairs(const gk_ctx *ctx, uint64_t np)
{
    uint64_t p = ctx->host_chunk_pairs;
    if (p == 0)
        p = std::min<uint64_t>(1u << 22, std::max<uint64_t>(1u << 20, (np + 15) / 16));
    p = std::min(p, np);
    return (p + 63) / 64 * 64;
}

}  // namespace

void gk_detail_free_host_pipe(gk_ctx *ctx)
{
    HostPipe &h = ctx->host;
    release(h.all);
    for (HostSlot &sl : h.slot) {
        release(sl.reads);
        release(sl.pair_read);
        release(sl.cand_pos);
        release(sl.e);
        release(sl.accept);
        release(sl.est);
        for (hipEvent_t *ev : {&sl.ev_in, &sl.ev_comp, &sl.ev_out}) {
            if (*ev)
                (void)hipEventDestroy(*ev);
            *ev = nullptr;
        }
    }
    for (hipEvent_t &ev : h.ev_read) {
        if (ev)
            (void)hipEventDestroy(ev);
        ev = nullptr;
    }
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
    gkd::TraceRange trace("gk_filter_host");
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
    const uint32_t rows = (b->max_read_len + 15) / 16;
    // ASCII reads encoded here on host threads (GK_OPT_HOST_ENCODE_THREADS):
    // 2-bit rows cross the bus, as for reads the caller encoded.
    const bool encode_here = !host_encoded && ctx->host_encode_threads > 0 && nr > 0;
    const bool rows_in = host_encoded || encode_here;
    const uint64_t text_bytes = (!host_encoded && nr) ? b->read_off[nr] : 0;
    const bool identity = b->pair_read == nullptr;
    constexpr uint32_t S = HostPipe::SLOTS;

    // Pair chunks of P pairs.  With pair i using read i, read chunk j is the
    // reads of pair chunk j and lives in slot j % S beside it; otherwise every
    // read stays resident (any pair may use any read), copied and encoded in
    // up to 16 chunks of R reads, and a pair chunk is filtered once the read
    // chunks holding its reads are encoded.
    const uint64_t P = chunk_pairs(ctx, np);
    const uint64_t K = (np + P - 1) / P;
    const uint64_t Kr = identity ? K : std::min<uint64_t>(K, 16);
    const uint64_t R = identity ? P : std::max<uint64_t>(1, (nr + Kr - 1) / Kr);
    // Transposed read words: pitch P in a slot, or every read in `all`.
    const uint32_t pitch =
        identity ? (uint32_t)P : (uint32_t)std::max<uint64_t>(64, (nr + 63) / 64 * 64);

    gk_detail_log(ctx, "gk_filter_host: %llu pairs, %llu reads, %s, chunks of %llu pairs "
                  "(%llu pair chunks, %llu read chunks, %u device slots), reads %s",
                  (unsigned long long)np, (unsigned long long)nr,
                  identity ? "one pair per read" : "pairs name their reads",
                  (unsigned long long)P, (unsigned long long)K, (unsigned long long)Kr, S,
                  host_encoded ? "host-encoded"
                               : (encode_here ? "encoded on host threads" : "encoded on the GPU"));
    HostPipe &h = ctx->host;
    hipError_t e = ensure_streams(h);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "streams and events");
    if (identity) {
        // A slot holds one read chunk's text from the 64-byte boundary at or
        // below its first offset, and 64 bytes of slack for aligned loads.
        uint64_t slot_text = 0;
        if (rows_in) {
            slot_text = P * rows * sizeof(uint32_t);
        } else {
            for (uint64_t j = 0; j < K; ++j) {
                const uint64_t r0 = std::min(nr, j * R), r1 = std::min(nr, r0 + R);
                const uint64_t a0 = b->read_off[r0] & ~63ull;
                const uint64_t a1 = std::min(b->read_off[r1], text_bytes);
                if (a1 > a0)
                    slot_text = std::max(slot_text, a1 - a0);
            }
            slot_text += 64;
        }
        for (uint32_t i = 0; i < S && i < K && e == hipSuccess; ++i)
            e = fit(h.slot[i].reads, slot_text, P, (uint64_t)rows * P);
    } else {
        e = fit(h.all, rows_in ? nr * rows * sizeof(uint32_t) : text_bytes + 64, nr,
                (uint64_t)rows * pitch);
    }
    for (uint32_t i = 0; i < S && i < K && e == hipSuccess; ++i) {
        HostSlot &sl = h.slot[i];
        e = fit(sl.cand_pos, P);
        if (e == hipSuccess && !identity)
            e = fit(sl.pair_read, P);
        if (e == hipSuccess && b->e)
            e = fit(sl.e, P);
        if (e == hipSuccess)
            e = fit(sl.accept, P);
        if (e == hipSuccess)
            e = fit(sl.est, P);
    }
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
                if ((e = gk_hmalloc((void **)&st, stage_bytes)) != hipSuccess)
                    return hip_fail(ctx, e, "pinned staging");
            h.stage_cap = stage_bytes;
        }
        if (h.pool_threads != ctx->host_encode_threads) {
            h.pool.reset();
            h.pool.reset(new gkd::HostEncodePool(ctx->host_encode_threads));
            h.pool_threads = ctx->host_encode_threads;
        }
    }

    // Last read chunk pair chunk q needs.  Pair chunks are considered in
    // order, so only the next one's is kept (found when it is first asked).
    uint64_t need_q = UINT64_MAX, need_val = 0;
    auto need_of = [&](uint64_t q) -> uint64_t {
        if (identity)
            return q;
        if (need_q != q) {
            const uint64_t q0 = q * P, q1 = std::min(np, q0 + P);
            uint32_t mx = 0;
            for (uint64_t i = q0; i < q1; ++i) {
                const uint32_t r = b->pair_read[i];
                if (r < nr && r > mx)
                    mx = r;          // pairs of reads >= n_reads are GK_INVALID
            }
            need_q = q;
            need_val = std::min<uint64_t>(Kr - 1, nr ? mx / R : 0);
        }
        return need_val;
    };

    // Pair chunk q: copies in, filter, copies out, in slot q % S.  Returns a
    // library status; hip errors land in e.
    auto run_pairs = [&](uint64_t q) -> int {
        HostSlot &sl = h.slot[q % S];
        const uint64_t q0 = q * P, q1 = std::min(np, q0 + P), n = q1 - q0;
        if (q >= S)          // the slot's inputs are free once chunk q - S is filtered
            e = hipStreamWaitEvent(h.s_in, sl.ev_comp, 0);
        if (e == hipSuccess)
            e = hipMemcpyAsync(sl.cand_pos.p, b->cand_pos + q0, n * sizeof(uint32_t),
                               hipMemcpyHostToDevice, h.s_in);
        if (e == hipSuccess && b->e)
            e = hipMemcpyAsync(sl.e.p, b->e + q0, n, hipMemcpyHostToDevice, h.s_in);
        if (e == hipSuccess && !identity)
            e = hipMemcpyAsync(sl.pair_read.p, b->pair_read + q0, n * sizeof(uint32_t),
                               hipMemcpyHostToDevice, h.s_in);
        if (e == hipSuccess)
            e = hipEventRecord(sl.ev_in, h.s_in);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(h.s_comp, sl.ev_in, 0);
        if (e == hipSuccess && q >= S)   // ... and its outputs once q - S is copied out
            e = hipStreamWaitEvent(h.s_comp, sl.ev_out, 0);
        if (e != hipSuccess)
            return GK_OK;
        gk_batch fb{};
        fb.pitch = pitch;
        fb.max_read_len = b->max_read_len;
        fb.e_uniform = b->e_uniform;
        fb.read_layout = host_encoded ? b->packed_layout : GK_READS_SPLIT;   // encode_here: split
        fb.flags = b->flags;
        fb.n_pairs = n;
        fb.cand_pos = sl.cand_pos.p;
        fb.e = b->e ? sl.e.p : nullptr;
        fb.accept = sl.accept.p;
        fb.est = sl.est.p;
        const HostReads &rd = identity ? sl.reads : h.all;
        fb.n_reads = identity ? (uint32_t)n : (uint32_t)nr;   // pair i of the chunk: read i
        fb.reads = rd.packed.p;
        fb.read_len = rd.len.p;
        fb.read_has_n = rd.has_n.p;
        fb.pair_read = identity ? nullptr : sl.pair_read.p;
        const int st = gk_filter(ctx, &fb, h.s_comp);
        if (st != GK_OK)
            return st;
        e = hipEventRecord(sl.ev_comp, h.s_comp);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(h.s_out, sl.ev_comp, 0);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->accept + q0, sl.accept.p, n, hipMemcpyDeviceToHost, h.s_out);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->est + q0, sl.est.p, n * sizeof(uint16_t),
                               hipMemcpyDeviceToHost, h.s_out);
        if (e == hipSuccess)
            e = hipEventRecord(sl.ev_out, h.s_out);
        return GK_OK;
    };

    int status = GK_OK;
    bool bad_offsets = false;
    uint64_t next_q = 0;
    for (uint64_t j = 0; j < Kr && e == hipSuccess && status == GK_OK; ++j) {
        // Read chunk j, into slot j % S (one pair per read) or into `all`.
        const uint64_t r0 = std::min(nr, j * R), r1 = std::min(nr, r0 + R), cnt = r1 - r0;
        HostReads &rd = identity ? h.slot[j % S].reads : h.all;
        const uint64_t at = identity ? 0 : r0;     // rd's index of read r0
        if (identity && j >= S)    // slot free once chunk j - S is filtered
            e = hipStreamWaitEvent(h.s_in, h.slot[j % S].ev_comp, 0);
        uint32_t *rows_dev =
            rows_in ? reinterpret_cast<uint32_t *>(rd.text.p) + at * rows : nullptr;
        uint64_t text_base = 0;
        if (e != hipSuccess || cnt == 0) {
            // nothing to copy (no reads left, or an error to report)
        } else if (encode_here) {
            for (uint64_t r = r0; r < r1 && !bad_offsets; ++r)
                bad_offsets = b->read_off[r + 1] < b->read_off[r];
            bad_offsets = bad_offsets || b->read_off[r1] > text_bytes;
            if (bad_offsets)
                break;
            if (j >= 2)
                e = hipEventSynchronize(h.ev_read[j & 1u]);
            uint8_t *st = h.stage[j & 1u];
            uint32_t *rows_h = reinterpret_cast<uint32_t *>(st);
            uint16_t *len_h = reinterpret_cast<uint16_t *>(st + stage_rows_bytes);
            uint8_t *has_n_h = st + stage_rows_bytes + R * sizeof(uint16_t);
            if (e == hipSuccess) {
                gkd::TraceRange trace_enc("gk_filter_host encode rows");
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
                e = hipMemcpyAsync(rd.len.p + at, len_h, cnt * sizeof(uint16_t),
                                   hipMemcpyHostToDevice, h.s_in);
            if (e == hipSuccess)
                e = hipMemcpyAsync(rd.has_n.p + at, has_n_h, cnt, hipMemcpyHostToDevice, h.s_in);
        } else if (host_encoded) {
            e = hipMemcpyAsync(rows_dev, b->packed + r0 * rows, cnt * rows * sizeof(uint32_t),
                               hipMemcpyHostToDevice, h.s_in);
            if (e == hipSuccess)
                e = hipMemcpyAsync(rd.len.p + at, b->read_len + r0, cnt * sizeof(uint16_t),
                                   hipMemcpyHostToDevice, h.s_in);
            if (e == hipSuccess)
                e = b->read_has_n
                        ? hipMemcpyAsync(rd.has_n.p + at, b->read_has_n + r0, cnt,
                                         hipMemcpyHostToDevice, h.s_in)
                        : hipMemsetAsync(rd.has_n.p + at, 0, cnt, h.s_in);
        } else {
            for (uint64_t r = r0; r < r1 && !bad_offsets; ++r)
                bad_offsets = b->read_off[r + 1] < b->read_off[r];
            bad_offsets = bad_offsets || b->read_off[r1] > text_bytes;
            if (bad_offsets)
                break;
            // The chunk's text: in a slot from the 64-byte boundary at or
            // below its first offset; in `all` at its own offsets.
            const uint64_t a0 = identity ? b->read_off[r0] & ~63ull : b->read_off[r0];
            const uint64_t a1 = b->read_off[r1];
            text_base = identity ? a0 : 0;
            if (a1 > a0)
                e = hipMemcpyAsync(rd.text.p + (a0 - text_base), b->ascii + a0, a1 - a0,
                                   hipMemcpyHostToDevice, h.s_in);
            // Offsets r0 .. r1; in `all`, offset r0 came with the previous
            // chunk, whose encoding may still be reading it.
            const uint64_t o0 = (identity || j == 0) ? r0 : r0 + 1;
            if (e == hipSuccess)
                e = hipMemcpyAsync(rd.off.p + at + (o0 - r0), b->read_off + o0,
                                   (r1 + 1 - o0) * sizeof(uint64_t), hipMemcpyHostToDevice,
                                   h.s_in);
        }
        if (e == hipSuccess)
            e = hipEventRecord(h.ev_read[j & 1u], h.s_in);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(h.s_comp, h.ev_read[j & 1u], 0);
        if (e == hipSuccess && cnt > 0)
            e = rows_in ? gkd::launch_transpose_reads(rows_dev, (uint32_t)cnt, rows, pitch,
                                                      rd.packed.p + at, h.s_comp)
                        : gkd::launch_encode_reads(rd.text.p, rd.off.p + at, (uint32_t)cnt, pitch,
                                                   rows, GK_READS_SPLIT, rd.packed.p + at,
                                                   rd.len.p + at, rd.has_n.p + at, h.s_comp,
                                                   text_base);
        // Every pair chunk whose reads are now encoded, in order.
        while (e == hipSuccess && status == GK_OK && next_q < K && need_of(next_q) <= j)
            status = run_pairs(next_q++);
    }
    gkd::trace_push("gk_filter_host drain");
    const hipError_t e1 = hipStreamSynchronize(h.s_in);
    const hipError_t e2 = hipStreamSynchronize(h.s_comp);
    const hipError_t e3 = hipStreamSynchronize(h.s_out);
    gkd::trace_pop();
    if (status != GK_OK)
        return status;
    if (e == hipSuccess)
        e = e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : e3);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "pipeline");
    if (bad_offsets)
        return fail(ctx, GK_EINVAL, "gk_filter_host: read_off decreases or passes the text end");
    ctx->err.clear();
    return GK_OK;
}

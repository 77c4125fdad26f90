// Internal declarations shared by the HIP sources of libgk (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "gk.h"
#include "gk_args.h"
#include "gk_host_encode.h"

// Tuning of the mixed-batch launch (never changes results).
struct MixedConfig {
    uint32_t tile = 4096;         // pairs per tile: 2048, 4096 or 8192
    uint32_t ppl = 1;             // pairs per lane per chunk: 1 or 2
    uint32_t sort_e = 1;          // sort a tile by (W, k_max) (1) or by W only (0)
    uint32_t blocks_per_cu = 0;   // persistent grid: 0 = as many as fit
};

// A device buffer of gk_filter_host and its capacity in elements.
template <typename T>
struct DevBuf {
    T *p = nullptr;
    uint64_t cap = 0;
};

// Reads on the device: their text (or host-encoded row-major words), offsets,
// lengths, unknown-base flags and transposed 2-bit words.
struct HostReads {
    DevBuf<uint8_t> text;
    DevBuf<uint64_t> off;
    DevBuf<uint16_t> len;
    DevBuf<uint8_t> has_n;
    DevBuf<uint32_t> packed;
};

// One chunk of gk_filter_host in flight: its pairs and results, and, when
// pair i uses read i, its reads.  ev_in: its copies in are done; ev_comp: its
// filter is done (inputs free); ev_out: its results are copied out (outputs
// free).
struct HostSlot {
    HostReads reads;
    DevBuf<uint32_t> pair_read, cand_pos;
    DevBuf<uint8_t> e, accept;
    DevBuf<uint16_t> est;
    hipEvent_t ev_in = nullptr, ev_comp = nullptr, ev_out = nullptr;
};

// Device buffers and streams of gk_filter_host, grown on demand and kept:
// SLOTS chunks in flight (copies in, filter, copies out), so device memory is
// bounded by the chunk size, plus every read of a batch whose pairs name
// their reads (any pair may use any read).
struct HostPipe {
    static constexpr uint32_t SLOTS = 3;
    hipStream_t s_in = nullptr, s_comp = nullptr, s_out = nullptr;
    HostSlot slot[SLOTS];
    HostReads all;
    hipEvent_t ev_read[2] = {nullptr, nullptr};   // read chunk j's copies: [j % 2]
    uint8_t *stage[2] = {nullptr, nullptr};   // pinned: host-encoded read chunks
    uint64_t stage_cap = 0;      // bytes of each
    std::unique_ptr<gkd::HostEncodePool> pool;  // host encoding threads
    unsigned pool_threads = 0;
};

struct gk_ctx {
    int device = 0;
    std::string err;
    uint64_t ref_len = 0;       // bases
    uint64_t ref_words = 0;     // ceil(ref_len / 32)
    uint64_t ref_unknown = 0;   // unknown bases
    uint2 *ref_planes = nullptr;
    uint2 *ref_planes_b = nullptr;            // planes shifted by half a line
    uint32_t *ref_unk = nullptr;
    unsigned long long *ref_unk_lines = nullptr;  // one bit per 512 bases
    unsigned long long *d_counter = nullptr;  // scratch for the unknown count
    uint32_t pairs_per_lane = 0;              // GK_OPT_PAIRS_PER_LANE
    int cu_count = 0;
    // mixed-batch launch
    MixedConfig mixed;
    uint32_t use_graph = 1;                   // GK_OPT_MIXED_GRAPH
    uint32_t host_encode_threads = 0;         // GK_OPT_HOST_ENCODE_THREADS
    uint64_t host_chunk_pairs = 0;            // GK_OPT_HOST_CHUNK_PAIRS (0: automatic)
    uint32_t log = 0;                         // GK_LOG: one stderr line per decision
    uint32_t autotune = 0;                    // GK_AUTOTUNE: AUTOTUNE_USE / _REFRESH / _OFF
    uint64_t server_part_pairs = 1u << 17;    // GK_OPT_SERVER_PART_PAIRS
    uint64_t server_tick_pairs = 1u << 20;    // GK_OPT_SERVER_TICK_PAIRS
    uint32_t server_copy_streams = 4;         // GK_OPT_SERVER_COPY_STREAMS
    uint32_t *d_mixed_counters = nullptr;     // [tile counter, residual count]
    uint32_t *d_resid = nullptr;              // residual pair list
    uint64_t resid_cap = 0;
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<uint8_t> graph_key;           // shape and tuning of graph_exec
    // the batch argument table the graph reads (device), and a ring of
    // pinned host copies it is filled from, each reusable once its event
    // (recorded after the graph launch that read it) has fired
    static constexpr int TABLE_RING = 4;
    gkd::BatchTable *d_table = nullptr;
    gkd::BatchTable *h_table[TABLE_RING] = {};
    hipEvent_t table_ev[TABLE_RING] = {};
    bool table_used[TABLE_RING] = {};
    uint32_t table_next = 0;
    HostPipe host;                            // gk_filter_host
    uint32_t *d_verify_list = nullptr;        // gk_verify: selected pairs (verify_cap
                                              // words), per-workgroup counts, deferred
                                              // pairs (verify_cap words)
    // d_verify_count: [0] selected pairs, [1] deferred pairs
    uint32_t *d_verify_count = nullptr;
    uint64_t verify_cap = 0;
    uint32_t *d_reads_rm = nullptr;           // gk_verify: row-major copy of the reads
    uint64_t reads_rm_cap = 0;                // (words)
};

// gk_tune_mixed's use of its cache (environment GK_AUTOTUNE=use|refresh|off):
// take a cached choice or measure and append (use), measure and append
// whatever the cache holds (refresh), or keep the context's tuning and time
// nothing (off).
constexpr uint32_t AUTOTUNE_USE = 0, AUTOTUNE_REFRESH = 1, AUTOTUNE_OFF = 2;

// One line "[gk] ..." on stderr when the context was created with GK_LOG=1:
// the choices a call makes (kernel, chunking, graph capture or replay, tuning).
void gk_detail_log(const gk_ctx *ctx, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

// Releases the buffers, streams and events of gk_filter_host.
void gk_detail_free_host_pipe(gk_ctx *ctx);

// Makes a device current for a scope and restores the caller's device.
struct DeviceScope {
    int prev = -1;
    bool ok = false;
    explicit DeviceScope(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess)
            prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceScope()
    {
        if (prev >= 0)
            (void)hipSetDevice(prev);
    }
};

// Every device and pinned-host allocation of the library goes through these
// two calls, so that gk_detail_fail_alloc can make the n-th one report
// hipErrorOutOfMemory (and allocate nothing) to test the error paths.
hipError_t gk_detail_device_alloc(void **p, size_t bytes);
hipError_t gk_detail_pinned_alloc(void **p, size_t bytes);

template <typename T>
hipError_t gk_dmalloc(T **p, size_t bytes)
{
    void *v = nullptr;
    const hipError_t e = gk_detail_device_alloc(&v, bytes);
    *p = static_cast<T *>(v);
    return e;
}

template <typename T>
hipError_t gk_hmalloc(T **p, size_t bytes)
{
    void *v = nullptr;
    const hipError_t e = gk_detail_pinned_alloc(&v, bytes);
    *p = static_cast<T *>(v);
    return e;
}

// Records msg as the context's last error and returns code.
inline int gk_detail_fail(gk_ctx *ctx, int code, const std::string &msg)
{
    if (ctx)
        ctx->err = msg;
    return code;
}

namespace gkd {

// Mixed-batch launch sequence: reset, persistent kernel, residual pass and
// (if a.accept_bits) the accept-bit pass, one set per 2^30 pairs.
hipError_t launch_mixed(const FilterArgs &a, const MixedArgs &x, uint32_t wmax, uint32_t layout,
                        hipStream_t s);
hipError_t mixed_blocks_per_cu(uint32_t wmax, uint32_t layout, uint32_t tile, uint32_t ppl,
                               int *out);
// Table launch sequence (reset, persistent kernel, residual pass) for the
// table at x.table; the tile count is read from the table on the device, so
// the sequence can be captured once and replayed with new table contents.
hipError_t launch_mixed_table(const MixedArgs &x, uint32_t wmax, uint32_t layout, hipStream_t s);
// Accept bits of n accept codes (bit j of word t: pair 64t + j is ACCEPT or
// UNDEFINED).
hipError_t launch_accept_bits(const uint8_t *accept, uint64_t n, unsigned long long *bits,
                              hipStream_t s);
size_t mixed_lds_size(uint32_t tile);

// Launch the filter that encodes its own reads (pair i uses read i, read i
// is ascii[read_off[i], read_off[i+1])), `words` 32-base words per mask.
hipError_t launch_filter_ascii(const FilterArgs &a, uint32_t words, const uint8_t *ascii,
                               const uint64_t *read_off, hipStream_t s);

// Launch the plain filter with `words` 32-base words per mask (1..16).
hipError_t launch_filter(const FilterArgs &a, uint32_t words, uint32_t layout,
                         uint32_t pairs_per_lane, hipStream_t s);

// Text offset t of read_off is at ascii[t - text_base]; text_base must not
// exceed read_off[0] (a chunk's text copied to the start of a buffer).
hipError_t launch_encode_reads(const uint8_t *ascii, const uint64_t *read_off, uint32_t n_reads,
                               uint32_t pitch, uint32_t rows, uint32_t layout, uint32_t *packed,
                               uint16_t *len_out, uint8_t *has_n_out, hipStream_t s,
                               uint64_t text_base = 0);

// Host-encoded reads, rows words per read in read order, to the transposed
// layout: out[w * pitch + r] = rowmajor[r * rows + w] for r < n_reads.
hipError_t launch_transpose_reads(const uint32_t *rowmajor, uint32_t n_reads, uint32_t rows,
                                  uint32_t pitch, uint32_t *out, hipStream_t s);

// Pack bases [first, first + n) of the reference, first a multiple of 32,
// from the device staging buffer `ascii` (holding those n bytes) into the
// resident planes; adds the number of unknown bases to *counter.
hipError_t launch_pack_reference(const uint8_t *ascii, uint64_t first, uint64_t n, uint2 *planes,
                                 uint32_t *unk, unsigned long long *counter, hipStream_t s);

}  // namespace gkd

// Internal declarations shared by the HIP sources of libgk (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "gk.h"

// Resident reference layout (device):
//   planes[j].x : bit b = high bit of the 2-bit code of base 32j+b
//   planes[j].y : bit b = low bit of the 2-bit code of base 32j+b
//   unknown[j]  : bit b = 1 iff base 32j+b is not A/C/G/T
// Bases at or beyond the reference length are 0 in all three.  REF_PAD_WORDS
// zero words follow the last word so that a window gather of up to
// GK_MAX_READ_LEN/32 + 1 words from any in-range window start stays inside
// the allocation.
namespace gkd {
constexpr uint32_t REF_PAD_WORDS = 32;
constexpr uint32_t MAX_WORDS = GK_MAX_READ_LEN / 32;  // 32-base words per mask
constexpr uint32_t GK_PPL_RESIDENT = 65536;  // pairs-per-lane value meaning
                                             // "one residency of the device"
}  // namespace gkd

// Tuning of the mixed-batch launch (never changes results).
struct MixedConfig {
    uint32_t tile = 4096;         // pairs per tile: 2048, 4096 or 8192
    uint32_t ppl = 1;             // pairs per lane per chunk: 1 or 2
    uint32_t sort_e = 1;          // sort a tile by (W, k_max) (1) or by W only (0)
    uint32_t blocks_per_cu = 0;   // persistent grid: 0 = as many as fit
};

struct gk_ctx {
    int device = 0;
    std::string err;
    uint64_t ref_len = 0;       // bases
    uint64_t ref_words = 0;     // ceil(ref_len / 32)
    uint64_t ref_unknown = 0;   // unknown bases
    uint2 *ref_planes = nullptr;
    uint32_t *ref_unk = nullptr;
    unsigned long long *d_counter = nullptr;  // scratch for the unknown count
    uint32_t pairs_per_lane = 0;              // GK_OPT_PAIRS_PER_LANE
    int cu_count = 0;
    // mixed-batch launch
    MixedConfig mixed;
    uint32_t use_graph = 1;                   // GK_OPT_MIXED_GRAPH
    uint32_t *d_mixed_counters = nullptr;     // [tile counter, residual count]
    uint32_t *d_resid = nullptr;              // residual pair list
    uint64_t resid_cap = 0;
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<uint8_t> graph_key;
};

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

// Records msg as the context's last error and returns code.
inline int gk_detail_fail(gk_ctx *ctx, int code, const std::string &msg)
{
    if (ctx)
        ctx->err = msg;
    return code;
}

namespace gkd {

struct FilterArgs {
    const uint2 *ref_planes;
    const uint32_t *ref_unk;
    uint64_t ref_len;
    uint32_t ref_has_unknown;
    uint32_t n_reads;
    uint32_t pitch;
    uint32_t e_uniform;
    uint32_t max_read_len;      // reads longer than this are GK_INVALID: the
                                // read rows hold ceil(max_read_len/16) words
    uint32_t rows;              // ceil(max_read_len / 16)
    uint32_t stream_reads;      // 1: every read and pair entry is used once
                                // (load them non-temporally), 0: reads are
                                // shared by several pairs (keep them cached)
    const uint32_t *reads;
    const uint16_t *read_len;
    const uint8_t *read_has_n;
    const uint32_t *pair_read;
    const uint32_t *cand_pos;
    const uint8_t *e_pair;
    uint64_t n_pairs;
    uint8_t *accept;
    uint16_t *est;
    unsigned long long *accept_bits;
};

// A table of batches filtered by one persistent launch (the serving loop's
// tick): batch b owns the launch's tiles [prefix[b], prefix[b+1]).
constexpr uint32_t MAX_TABLE_BATCHES = 256;
struct BatchTable {
    uint32_t n_batches;
    uint32_t pad_[3];
    uint32_t prefix[MAX_TABLE_BATCHES + 1];
    FilterArgs args[MAX_TABLE_BATCHES];
};

struct MixedArgs {
    const BatchTable *table;     // device table, or nullptr for the single batch
    uint32_t *tile_counter;      // zeroed by the launch sequence
    uint32_t *resid_count;       // zeroed by the launch sequence
    uint32_t *resid_list;        // capacity >= pairs per launch
    uint32_t n_tiles;            // set per launch
    uint32_t tile;               // pairs per tile (multiple of 256, <= 8192)
    uint32_t ppl;                // 1 or 2
    uint32_t sort_e;             // 0 or 1
    uint32_t blocks;             // persistent workgroups
    uint32_t resid_blocks;       // grid of the residual pass
};

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
size_t mixed_lds_size(uint32_t tile);

// Launch the plain filter with `words` 32-base words per mask (1..16).
hipError_t launch_filter(const FilterArgs &a, uint32_t words, uint32_t layout,
                         uint32_t pairs_per_lane, hipStream_t s);

hipError_t launch_encode_reads(const uint8_t *ascii, const uint64_t *read_off, uint32_t n_reads,
                               uint32_t pitch, uint32_t rows, uint32_t layout, uint32_t *packed,
                               uint16_t *len_out, uint8_t *has_n_out, hipStream_t s);

// Pack bases [first, first + n) of the reference, first a multiple of 32,
// from the device staging buffer `ascii` (holding those n bytes) into the
// resident planes; adds the number of unknown bases to *counter.
hipError_t launch_pack_reference(const uint8_t *ascii, uint64_t first, uint64_t n, uint2 *planes,
                                 uint32_t *unk, unsigned long long *counter, hipStream_t s);

}  // namespace gkd

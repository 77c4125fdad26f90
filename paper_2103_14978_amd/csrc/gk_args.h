// Kernel-facing declarations of libgk: the resident reference layout and the
// argument blocks the filter kernels take (host-only state is in
// gk_internal.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

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

// Second copy of the planes, shifted by half a 128-byte cache line:
// ref_planes_b[j] = ref_planes[j + REF_SHIFT_WORDS].  A window gather of up to
// 9 words that crosses a line of ref_planes lies within one line of
// ref_planes_b, so every window of up to 256 bases costs one line fetch.
constexpr uint32_t LINE_WORDS = 16;          // uint2 words per 128-byte line
constexpr uint32_t LINE_BASES = 32 * LINE_WORDS;
constexpr uint32_t REF_SHIFT_WORDS = 8;

struct FilterArgs {
    const uint2 *ref_planes;
    const uint2 *ref_planes_b;  // ref_planes shifted by REF_SHIFT_WORDS, or NULL
    const uint32_t *ref_unk;
    const unsigned long long *ref_unk_lines;  // bit L: bases [512 L, 512 L + 512)
                                              // hold an unknown base
    uint64_t ref_len;
    uint32_t ref_has_unknown;
    uint32_t n_reads;
    uint32_t pitch;
    uint32_t e_uniform;
    uint32_t max_read_len;      // reads longer than this are GK_INVALID: the
                                // read rows hold ceil(max_read_len/16) words
    uint32_t rows;              // ceil(max_read_len / 16)
    uint32_t flags;             // GK_FLAG_* variant semantics (0: the paper's)
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

}  // namespace gkd

// Internal declarations shared by the HIP sources of libgk (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

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
}  // namespace gkd

struct gk_ctx {
    int device = 0;
    std::string err;
    uint64_t ref_len = 0;       // bases
    uint64_t ref_words = 0;     // ceil(ref_len / 32)
    uint64_t ref_unknown = 0;   // unknown bases
    uint2 *ref_planes = nullptr;
    uint32_t *ref_unk = nullptr;
    unsigned long long *d_counter = nullptr;  // scratch for the unknown count
};

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

// Launch the plain filter with `words` 32-base words per mask (1..16).
hipError_t launch_filter(const FilterArgs &a, uint32_t words, hipStream_t s);

hipError_t launch_encode_reads(const uint8_t *ascii, const uint64_t *read_off, uint32_t n_reads,
                               uint32_t pitch, uint32_t rows, uint32_t *packed, uint16_t *len_out,
                               uint8_t *has_n_out, hipStream_t s);

// Pack bases [first, first + n) of the reference, first a multiple of 32,
// from the device staging buffer `ascii` (holding those n bytes) into the
// resident planes; adds the number of unknown bases to *counter.
hipError_t launch_pack_reference(const uint8_t *ascii, uint64_t first, uint64_t n, uint2 *planes,
                                 uint32_t *unk, unsigned long long *counter, hipStream_t s);

}  // namespace gkd

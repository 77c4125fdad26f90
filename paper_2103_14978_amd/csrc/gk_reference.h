// Launchers that build the resident reference from a caller's 2-bit words
// (the ASCII path is launch_pack_reference in gk_internal.h).
#pragma once

#include "gk_internal.h"

namespace gkd {

// Planes of bases [first, first + n), first a multiple of 32, from the device
// staging buffer `packed` holding ceil(n / 16) words of 16 bases each in
// `layout`.  Code bits at or beyond n are cleared.
hipError_t launch_unpack_reference(const uint32_t *packed, uint64_t first, uint64_t n,
                                   uint32_t layout, uint2 *planes, hipStream_t s);

// Sets the unknown-base bits of n_runs (start, length) pairs held in device
// memory; runs may overlap and lie in bases [0, ref_len).
hipError_t launch_mark_runs(const uint64_t *runs, uint64_t n_runs, uint32_t *unk, hipStream_t s);

// Adds the number of set bits of unk[0, words) to *counter.
hipError_t launch_count_unknown(const uint32_t *unk, uint64_t words, unsigned long long *counter,
                                hipStream_t s);

// lines[L / 64] bit L % 64 = 1 iff unknown-plane words [16 L, 16 L + 16) hold a
// set bit; `lines` has ceil(ceil(words / 16) / 64) entries.
hipError_t launch_unknown_lines(const uint32_t *unk, uint64_t words, unsigned long long *lines,
                                hipStream_t s);

}  // namespace gkd

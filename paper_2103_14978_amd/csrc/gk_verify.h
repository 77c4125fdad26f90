// Launcher of the verification kernels (gk_verify).
#pragma once

#include "gk_args.h"

namespace gkd {

// dist[i] = min(edit distance, e_i + 1) for the pairs with accept[i] ==
// GK_ACCEPT (every pair when accept is NULL); GK_EST_NONE for the others and
// for pairs that cannot be compared or have e_i > GK_VERIFY_MAX_E.  list,
// groups, deferred and count are scratch: min(n_pairs, 2^30) words, one word
// per 4096 of those pairs (rounded up), min(n_pairs, 2^30) words and two
// words; bins: VERIFY_BIN_WORDS words (the listing by length and e of a
// batch with a per-pair e).  reads_rm: NULL, or scratch of
// n_reads * verify_rm_stride(rows) words for a row-major copy of the reads,
// which the one-pair-per-lane kernel then reads its pairs' words from.
hipError_t launch_verify(const FilterArgs &a, const uint8_t *accept, uint16_t *dist,
                         uint32_t *list, uint32_t *groups, uint32_t *deferred, uint32_t *count,
                         uint32_t *bins, uint32_t *reads_rm, uint32_t words, uint32_t layout,
                         int cus, hipStream_t s);

constexpr uint32_t VERIFY_BIN_WORDS = 3u * 512u * 32u;

// Words per read of the row-major copy: rows rounded up to a multiple of 4.
inline uint32_t verify_rm_stride(uint32_t rows) { return (rows + 3u) & ~3u; }

}  // namespace gkd

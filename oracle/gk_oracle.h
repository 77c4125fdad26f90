/*
 * GateKeeper-GPU oracle: plain, slow, per-base CPU implementation of the
 * pre-alignment filter described in "GateKeeper-GPU: Fast and Accurate
 * Pre-Alignment Filtering in Short Read Mapping" (Bingol et al., 2021).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the product path.
 * Only tests, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  It shares no code, header, table or helper with the HIP library.
 *
 * Every function works on plain ASCII strings, one base at a time, in the
 * order the paper gives the steps; there is no bit packing and no blocking.
 */
#ifndef GK_ORACLE_H
#define GK_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* Result codes per pair. */
#define GKO_REJECT    0u   /* edit estimate exceeds e                        */
#define GKO_ACCEPT    1u   /* edit estimate <= e                             */
#define GKO_UNDEFINED 2u   /* unknown base or window past the reference end:
                              passed without filtering (Sec. 3.3)             */
#define GKO_INVALID   3u   /* read length 0 or above GKO_MAX_LEN             */
#define GKO_EST_NONE  0xFFFFu
#define GKO_MAX_LEN   512u

/* Flags. */
#define GKO_NO_REFINE 1u   /* skip the leading/trailing refinement (Sec. 3.4):
                              the original GateKeeper behaviour               */
#define GKO_HAMMING_FASTPATH 2u /* a variant the paper does not describe: a
                              pair whose Hamming distance (count of differing
                              codes) is at most e is accepted with that count
                              as its estimate; otherwise the masks decide     */

/* Stages recorded by gko_filter_pair_trace, per mask. */
#define GKO_STAGE_RAW     0
#define GKO_STAGE_AMENDED 1
#define GKO_STAGE_REFINED 2

/* Amend one mask (Sec. 2.1): every maximal run of 0s of length 1 or 2 that
   has a 1 on both sides inside [0, m) becomes 1s.  Runs that touch position 0
   or m-1 are left alone.  in/out hold one byte (0/1) per position; they may
   alias.  Returns 0. */
int gko_amend(const uint8_t *in, uint32_t m, uint8_t *out);

/* Filter one pair: read[0..m) against ref[pos .. pos+m) with threshold e.
   Returns one of the GKO_* result codes and stores the edit estimate in *est
   (GKO_EST_NONE unless the result is REJECT or ACCEPT). */
uint32_t gko_filter_pair(const char *read, uint32_t m, const char *ref,
                         uint64_t ref_len, uint64_t pos, uint32_t e,
                         uint32_t flags, uint16_t *est);

/* Same, and also records every mask.  masks must hold
   (2*e_eff + 1) * 3 * m bytes where e_eff = min(e, m); mask slot s is
   d = 0 for s = 0, d = +k (deletion) for s = 2k-1, d = -k (insertion) for
   s = 2k; each slot holds stages RAW, AMENDED, REFINED of m bytes each.
   Slots are written only when the result is REJECT or ACCEPT and the Hamming
   fast path (if asked for) did not decide. */
uint32_t gko_filter_pair_trace(const char *read, uint32_t m, const char *ref,
                               uint64_t ref_len, uint64_t pos, uint32_t e,
                               uint32_t flags, uint16_t *est, uint8_t *masks);

/* Batch driver: pair i compares read pair_read[i] (ASCII at
   reads + read_off[r], length read_off[r+1]-read_off[r]) with the window at
   cand_pos[i].  e_pair may be NULL (then e_uniform applies).  n_threads >= 1
   splits the pairs into contiguous ranges, one POSIX thread each. */
int gko_filter_batch(const char *reads, const uint64_t *read_off,
                     uint32_t n_reads, const char *ref, uint64_t ref_len,
                     const uint32_t *pair_read, const uint32_t *cand_pos,
                     const uint8_t *e_pair, uint32_t e_uniform,
                     uint64_t n_pairs, uint32_t flags, uint32_t n_threads,
                     uint8_t *accept, uint16_t *est);

/* Global edit (Levenshtein) distance with unit costs between a[0..n) and
   b[0..p), capped: returns min(distance, cap + 1).  Computes only the cells
   within `cap` of the main diagonal when cap < max(n, p). */
uint32_t gko_levenshtein(const char *a, uint32_t n, const char *b, uint32_t p,
                         uint32_t cap);

/* Full O(n*p) dynamic program, no band: the textbook definition. */
uint32_t gko_levenshtein_full(const char *a, uint32_t n, const char *b,
                              uint32_t p);

/* Batch Levenshtein over the same pair description as gko_filter_batch;
   windows past the reference end get cap + 1. */
int gko_levenshtein_batch(const char *reads, const uint64_t *read_off,
                          uint32_t n_reads, const char *ref, uint64_t ref_len,
                          const uint32_t *pair_read, const uint32_t *cand_pos,
                          uint64_t n_pairs, uint32_t cap, uint32_t n_threads,
                          uint16_t *dist);

#ifdef __cplusplus
}
#endif
#endif

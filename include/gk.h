/*
 * gk.h — C ABI of the MI355X (gfx950) GateKeeper-GPU pre-alignment filter.
 *
 * The filter is the one of "GateKeeper-GPU: Fast and Accurate Pre-Alignment
 * Filtering in Short Read Mapping" (Bingol, Alser, Mutlu, Ozturk, Alkan):
 * for each (read, candidate reference position, error threshold e) it builds
 * the Hamming mask and the 2e shifted deletion/insertion masks from the 2-bit
 * encodings (Sec. 2.1), amends short 0-streaks in every mask, sets each
 * shifted mask's vacated leading/trailing bits to 1 (Sec. 3.4), ANDs the
 * 2e+1 masks, counts the surviving 1s as the edit estimate and accepts the
 * pair iff that count is <= e.  Pairs holding an unknown base pass without
 * filtering (Sec. 3.3).
 *
 * Conventions for every function:
 *   - Return value: GK_OK (0) or a negative GK_E* code.  Nothing is thrown
 *     across the ABI.  gk_last_error() gives a message for the last failure.
 *   - "device" pointers are HIP device allocations on the context's GPU;
 *     "host" pointers are ordinary process memory.  The caller owns every
 *     buffer it passes; the context owns the resident reference.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).
 *     Functions that take a stream only enqueue work and return; completion
 *     is the caller's stream synchronisation.  Buffers must stay alive until
 *     that work completes.
 *   - Per-pair data problems never fail a call: they show up per pair as
 *     GK_UNDEFINED or GK_INVALID (see below).
 *   - A gk_ctx is not thread-safe: one thread at a time per context.
 *   - A device fault returns GK_EDEVICE; the context must then be destroyed.
 */
#ifndef GK_H
#define GK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define GK_OK        0
#define GK_EINVAL   (-1)   /* bad argument (NULL, size, range)               */
#define GK_ENOMEM   (-2)   /* device or host allocation failed               */
#define GK_EDEVICE  (-3)   /* HIP runtime or device error                    */
#define GK_ENOREF   (-4)   /* no reference loaded                            */
#define GK_ERANGE   (-5)   /* size beyond a documented limit                 */

/* Per-pair result codes written to gk_batch.accept. */
#define GK_REJECT     0u   /* edit estimate > e                              */
#define GK_ACCEPT     1u   /* edit estimate <= e                             */
#define GK_UNDEFINED  2u   /* read or window holds a base other than A/C/G/T,
                              or the window runs past the reference end:
                              passed without filtering (Sec. 3.3)             */
#define GK_INVALID    3u   /* read length 0, above max_read_len, or read
                              index out of range                             */

#define GK_EST_NONE      0xFFFFu  /* est of UNDEFINED / INVALID pairs        */
#define GK_MAX_READ_LEN  512u     /* longest read the kernels take           */
#define GK_MAX_REF_LEN   0xFFFFFFFFull /* positions are 32-bit               */

typedef struct gk_ctx gk_ctx;

/* Create a context on HIP device `device`.  *out is set on success. */
int gk_create(int device, gk_ctx **out);

/* Free the context, its resident reference and scratch.  NULL-safe. */
void gk_destroy(gk_ctx *ctx);

/* Message for the last failing call on ctx (never NULL; "" if none).  With
   ctx == NULL: the message of the last failing gk_create in this thread. */
const char *gk_last_error(const gk_ctx *ctx);

/*
 * Reference residency (Sec. 3.5: the reference is encoded once and the
 * positions of unknown bases are recorded).
 *
 * ascii: HOST pointer to len bytes.  A/C/G/T in either case are bases; every
 * other byte is an unknown base.  The reference is 2-bit encoded on the GPU
 * (A=00 C=01 G=10 T=11, Sec. 2.1) and kept resident until the context is
 * destroyed or another reference replaces it.  Synchronous: returns after the
 * device copy is complete.  len must be 1..GK_MAX_REF_LEN (else GK_ERANGE /
 * GK_EINVAL).  On failure the previous reference (if any) is dropped.
 */
int gk_load_reference(gk_ctx *ctx, const char *ascii, uint64_t len);

/* Length and number of unknown bases of the resident reference. */
int gk_reference_info(const gk_ctx *ctx, uint64_t *len, uint64_t *n_unknown);

/*
 * Read encoding (Sec. 3.3: reads are 2-bit encoded, 16 bases per 32-bit word).
 *
 * ascii, read_off: DEVICE.  Read r is ascii[read_off[r] .. read_off[r+1]),
 * read_off has n_reads + 1 entries.
 * packed_out: DEVICE, rows * pitch words.  Word w of read r is written at
 * packed_out[w * pitch + r] (transposed, so a wavefront's loads coalesce):
 * base i of the read sits in bits 2(i mod 16), 2(i mod 16)+1 of word i / 16
 * (least-significant first); bits at or beyond twice the read length are 0,
 * words at or beyond ceil(len / 16) are 0.  Bases beyond 16 * rows are
 * dropped (give rows >= ceil(max length / 16)).
 * len_out: DEVICE, n_reads entries: the read length (capped at 0xFFFF).
 * has_n_out: DEVICE, n_reads entries or NULL: 1 if the read holds a byte other
 * than A/C/G/T (either case) within its first 16 * rows bytes, else 0.
 * Requires pitch >= n_reads, 1 <= rows <= 32.  Asynchronous on stream.
 */
int gk_encode_reads(gk_ctx *ctx, const uint8_t *ascii, const uint64_t *read_off,
                    uint32_t n_reads, uint32_t pitch, uint32_t rows,
                    uint32_t *packed_out, uint16_t *len_out, uint8_t *has_n_out,
                    void *stream);

/*
 * A batch of pairs.  All pointers are DEVICE pointers owned by the caller.
 * Pair i compares read pair_read[i] (length read_len[r]) with the reference
 * window ref[cand_pos[i], cand_pos[i] + read_len[r]) under threshold e_i
 * (e[i], or e_uniform when e == NULL).
 */
typedef struct gk_batch {
    uint32_t        n_reads;
    uint32_t        pitch;         /* >= n_reads: row stride of reads        */
    uint32_t        max_read_len;  /* 1..GK_MAX_READ_LEN, host-side bound on
                                      every read_len[r]; picks the kernel's
                                      words per mask.  Reads longer than it
                                      give GK_INVALID pairs.                 */
    uint32_t        e_uniform;     /* threshold when e == NULL, 0..255       */
    const uint32_t *reads;         /* packed 2-bit transposed, the layout
                                      gk_encode_reads writes; needs
                                      ceil(max_read_len/16) rows             */
    const uint16_t *read_len;      /* n_reads entries                        */
    const uint8_t  *read_has_n;    /* n_reads entries, or NULL (no unknowns) */
    uint64_t        n_pairs;
    const uint32_t *pair_read;     /* n_pairs: read index of each pair       */
    const uint32_t *cand_pos;      /* n_pairs: 0-based window start          */
    const uint8_t  *e;             /* n_pairs thresholds, or NULL            */
    uint8_t        *accept;        /* out, n_pairs: GK_REJECT .. GK_INVALID  */
    uint16_t       *est;           /* out, n_pairs: edit estimate (count of
                                      1s in the final mask) for REJECT and
                                      ACCEPT pairs, GK_EST_NONE otherwise     */
    uint64_t       *accept_bits;   /* out or NULL, ceil(n_pairs/64) words:
                                      bit (i mod 64) of word i/64 is 1 iff
                                      pair i is ACCEPT or UNDEFINED (i.e. it
                                      goes on to verification)               */
} gk_batch;

/*
 * Plain filter: one launch over all pairs of the batch, one GPU lane per pair
 * (Sec. 3.2: one thread per filtration), the read and window held as 32-base
 * bit-planes in registers.  Asynchronous on stream.
 * Errors (nothing launched): GK_EINVAL for NULL required pointers, pitch <
 * n_reads, max_read_len outside 1..512, e_uniform > 255; GK_ENOREF without a
 * reference; GK_ERANGE for n_pairs >= 2^38.
 */
int gk_filter(gk_ctx *ctx, const gk_batch *batch, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* GK_H */

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
#define GK_ETIMEOUT (-7)   /* gk_server_wait: not finished within the timeout */
#define GK_ECANCELED (-8)  /* request cancelled by gk_server_stop before it
                              was admitted                                   */

/* Per-pair result codes written to gk_batch.accept. */
#define GK_REJECT     0u   /* edit estimate > e                              */
#define GK_ACCEPT     1u   /* edit estimate <= e                             */
#define GK_UNDEFINED  2u   /* read or window holds a base other than A/C/G/T,
                              or the window runs past the reference end:
                              passed without filtering (Sec. 3.3)             */
#define GK_INVALID    3u   /* read length 0, above max_read_len, or read
                              index out of range                             */

#define GK_EST_NONE      0xFFFFu  /* est of UNDEFINED / INVALID pairs        */

/* Layouts of 2-bit encoded reads (A=00 C=01 G=10 T=11, Sec. 2.1): 16 bases
   per 32-bit word, base i of a read in word i / 16 at j = i mod 16.        */
#define GK_READS_SPLIT        0u  /* low code bit at bit j, high code bit at
                                     bit 16 + j (the filter's native form)   */
#define GK_READS_INTERLEAVED  1u  /* code at bits 2j (low) and 2j+1 (high)   */
#define GK_MAX_READ_LEN  512u     /* longest read the kernels take           */
#define GK_MAX_REF_LEN   0xFFFFFFFFull /* positions are 32-bit               */
#define GK_NOALLOC_MAX_PAIRS 4194304u /* pairs per gk_filter_mixed_noalloc call */

typedef struct gk_ctx gk_ctx;

/* Create a context on HIP device `device`.  *out is set on success.  Tuning
   options set in the environment (GK_<name>, see gk_set_option) apply to it;
   GK_EINVAL for a malformed one. */
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

/*
 * Reference residency from a 2-bit reference the caller already holds
 * (Sec. 3.3 fixes 16 bases per 32-bit word; Sec. 3.5 records the unknown
 * positions beside the codes).
 *
 * packed: HOST pointer to ceil(len / 16) words.  Base i is in word i / 16 at
 * j = i mod 16, with codes A=00 C=01 G=10 T=11 (Sec. 2.1), laid out as
 * `layout`: GK_READS_SPLIT (low code bit at bit j, high bit at bit 16 + j) or
 * GK_READS_INTERLEAVED (code at bits 2j, 2j + 1).  Code bits at or beyond len
 * are ignored.
 * n_runs: HOST pointer to n_n_runs (start, length) pairs of uint64, or NULL
 * when n_n_runs is 0: the bases in [start, start + length) are unknown (their
 * codes are ignored).  Runs may be in any order and may overlap; a run of
 * length 0 is ignored; a run reaching past len is an error.
 * Synchronous, like gk_load_reference, and gives the same resident state as
 * gk_load_reference on the matching ASCII text.  len must be
 * 1..GK_MAX_REF_LEN (GK_ERANGE above).  Argument errors (GK_EINVAL,
 * GK_ERANGE) are found before anything changes and keep the previous
 * reference; a device failure drops it.
 */
int gk_load_reference_2bit(gk_ctx *ctx, const uint32_t *packed, uint64_t len, uint32_t layout,
                           const uint64_t *n_runs, uint64_t n_n_runs);

/* Length and number of unknown bases of the resident reference. */
int gk_reference_info(const gk_ctx *ctx, uint64_t *len, uint64_t *n_unknown);

/*
 * Read encoding (Sec. 3.3: reads are 2-bit encoded, 16 bases per 32-bit word).
 *
 * ascii, read_off: DEVICE.  Read r is ascii[read_off[r] .. read_off[r+1]),
 * read_off has n_reads + 1 entries; a read whose end offset is below its
 * start is empty (length 0).  The text is read in aligned 4-byte words, so
 * the rest of the word that holds a read's last byte may be read (never
 * past that word).
 * packed_out: DEVICE, rows * pitch words.  Word w of read r is written at
 * packed_out[w * pitch + r] (transposed, so a wavefront's loads coalesce)
 * and holds bases 16w .. 16w+15 in the given layout (GK_READS_*); code bits
 * of positions at or beyond the read length are 0, words at or beyond
 * ceil(len / 16) are 0.  Bases beyond 16 * rows are dropped (give rows >=
 * ceil(max length / 16)).
 * len_out: DEVICE, n_reads entries: the read length (capped at 0xFFFF).
 * has_n_out: DEVICE, n_reads entries or NULL: 1 if the read holds a byte other
 * than A/C/G/T (either case) within its first 16 * rows bytes, else 0.
 * Requires n_reads < 2^30, pitch >= n_reads, pitch < 2^30, 1 <= rows <= 32,
 * layout GK_READS_SPLIT or GK_READS_INTERLEAVED.  Asynchronous on stream.
 */
int gk_encode_reads(gk_ctx *ctx, const uint8_t *ascii, const uint64_t *read_off,
                    uint32_t n_reads, uint32_t pitch, uint32_t rows, uint32_t layout,
                    uint32_t *packed_out, uint16_t *len_out, uint8_t *has_n_out,
                    void *stream);

/*
 * Variant semantics of a batch (gk_batch.flags, gk_host_batch.flags).  The
 * default, 0, is GateKeeper-GPU as the paper gives it.
 * GK_FLAG_NO_REFINE: skip the leading/trailing refinement of the shifted
 *   masks (Sec. 3.4), which gives the original GateKeeper's results.
 * GK_FLAG_HAMMING_FASTPATH: a variant the paper does not describe: a pair
 *   whose Hamming distance (count of differing bases) is at most e is
 *   accepted with that count as its estimate; other pairs go through the
 *   masks as usual.
 */
#define GK_FLAG_NO_REFINE        1u
#define GK_FLAG_HAMMING_FASTPATH 2u

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
    uint32_t        read_layout;   /* GK_READS_SPLIT or GK_READS_INTERLEAVED */
    const uint32_t *reads;         /* 2-bit encoded, 16 bases per word,
                                      transposed as gk_encode_reads writes
                                      them; ceil(max_read_len/16) rows of
                                      pitch words                            */
    const uint16_t *read_len;      /* n_reads entries                        */
    const uint8_t  *read_has_n;    /* n_reads entries, or NULL (no unknowns) */
    uint64_t        n_pairs;
    const uint32_t *pair_read;     /* n_pairs: read index of each pair, or
                                      NULL: pair i uses read i              */
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
    uint32_t        flags;         /* 0 (the paper's filter) or an OR of
                                      GK_FLAG_NO_REFINE and
                                      GK_FLAG_HAMMING_FASTPATH               */
} gk_batch;

/*
 * Plain filter: one kernel launch over all pairs of the batch (one launch per
 * 2^30 pairs), one GPU lane per pair at a time (Sec. 3.2: one thread per
 * filtration), the read and window held as 32-base bit-planes in registers.
 * Asynchronous on stream.
 * Errors (nothing launched): GK_EINVAL for NULL required pointers, pitch <
 * n_reads, n_reads or pitch >= 2^30, max_read_len outside 1..512, e_uniform
 * > 255, an unknown read_layout; GK_ENOREF without a reference; GK_ERANGE
 * for n_pairs >= 2^38.
 */
int gk_filter(gk_ctx *ctx, const gk_batch *batch, void *stream);

/*
 * Filter that encodes its reads in the same launch: the paper's
 * device-encoded mode, where the kernel encodes the sequences it is handed
 * in ASCII (Sec. 3.3; the device-encoded rows of Table 2).  Pair i compares
 * read i (one candidate per read) with ref[cand_pos[i], cand_pos[i] + m);
 * the 2-bit reads are never written to memory.
 *
 * batch: as for gk_filter, except that pair_read must be NULL and the read
 * fields (n_reads, pitch, reads, read_len, read_has_n, read_layout) are not
 * used.
 * ascii: DEVICE, 16-byte aligned.  Read i is ascii[read_off[i] ..
 * read_off[i+1]); read_off: DEVICE, n_pairs + 1 entries.  The launch reads
 * the text in aligned 4-byte words, so it may read the rest of the word that
 * holds a read's last byte (never past that word).  As for
 * gk_encode_reads, an end offset below the start gives an empty read, a
 * read's length is capped at 0xFFFF, and a byte other
 * than A/C/G/T (either case) in a read of length 1..max_read_len makes its
 * pair GK_UNDEFINED.
 * Results and accept bits equal those of gk_encode_reads (split layout,
 * rows = ceil(max_read_len / 16)) followed by gk_filter on the same reads.
 * Asynchronous on stream.  Errors as gk_filter, plus GK_EINVAL for a
 * non-NULL pair_read, a NULL ascii or read_off, or an unaligned ascii.
 */
int gk_filter_ascii(gk_ctx *ctx, const gk_batch *batch, const uint8_t *ascii,
                    const uint64_t *read_off, void *stream);

/*
 * Host-to-host filter: the whole path from reads in host memory to results
 * in host memory (the paper's filter time, Sec. 4.3, as opposed to kernel
 * time), with the host-to-device copies, the read encoding (Sec. 3.3, on the
 * GPU), the filter and the device-to-host copies of successive chunks of the
 * batch overlapped on three streams.
 *
 * All pointers are HOST pointers owned by the caller.  Copies overlap with
 * the kernels only when the buffers are pinned (hipHostMalloc); pageable
 * memory gives the same results.  Read r is ascii[read_off[r] ..
 * read_off[r+1]); read_off has n_reads + 1 non-decreasing entries and
 * read_off[0] == 0.  Pair i compares read pair_read[i] (pair_read NULL: read
 * i, and then n_pairs == n_reads) with ref[cand_pos[i], cand_pos[i] + m)
 * under e[i] (or e_uniform when e is NULL); accept[i] and est[i] are as in
 * gk_filter.  The device buffers are the context's, kept for later calls and
 * freed with it.  The chunks (GK_OPT_HOST_CHUNK_PAIRS pairs each) cycle
 * through three device slots, so device memory is bounded by the chunk size:
 * about 3 * chunk * (19 + 4 * ceil(max_read_len / 16) + mean read length)
 * bytes with pair_read NULL.  With pair_read, any pair may use any read, so
 * every read stays on the device (its text or rows plus its 2-bit words),
 * and the pairs take 3 * chunk * 12 bytes.
 * Synchronous: returns once every result is in host memory.  Errors:
 * GK_EINVAL for NULL buffers, read_off[0] != 0, decreasing offsets (found
 * while the batch is in flight: the outputs are then unspecified),
 * n_reads >= 2^30, or max_read_len outside 1..GK_MAX_READ_LEN; GK_ENOREF
 * without a reference; GK_ENOMEM when the device buffers do not fit.
 *
 * Host-encoded reads (the paper's host-encoded mode, Sec. 3.3): when packed
 * is not NULL, ascii and read_off are ignored and the reads come already
 * 2-bit encoded: read r's rows = ceil(max_read_len / 16) words are
 * packed[r * rows .. r * rows + rows), 16 bases per word in packed_layout
 * (GK_READS_SPLIT or GK_READS_INTERLEAVED, as gk_encode_reads writes them),
 * with every code bit at or beyond read_len[r] equal to 0.  read_len (HOST,
 * n_reads) is then required, read_has_n (HOST, n_reads, 1 = the read holds an
 * unknown base) is optional.  The GPU transposes the rows into the filter's
 * layout; about a quarter of the ASCII bytes cross PCIe.
 */
typedef struct gk_host_batch {
    uint32_t        n_reads;
    uint32_t        max_read_len;  /* 1..GK_MAX_READ_LEN (longer reads give
                                      GK_INVALID pairs)                      */
    const uint8_t  *ascii;         /* HOST reads, ASCII                      */
    const uint64_t *read_off;      /* HOST, n_reads + 1 entries              */
    uint64_t        n_pairs;
    const uint32_t *pair_read;     /* HOST n_pairs, or NULL                  */
    const uint32_t *cand_pos;      /* HOST n_pairs                           */
    const uint8_t  *e;             /* HOST n_pairs, or NULL                  */
    uint32_t        e_uniform;     /* 0..255                                 */
    uint8_t        *accept;        /* HOST out, n_pairs                      */
    uint16_t       *est;           /* HOST out, n_pairs                      */
    uint32_t        flags;         /* GK_FLAG_*, as gk_batch.flags           */
    const uint32_t *packed;        /* HOST host-encoded reads, or NULL       */
    const uint16_t *read_len;      /* HOST n_reads (with packed)             */
    const uint8_t  *read_has_n;    /* HOST n_reads or NULL (with packed)     */
    uint32_t        packed_layout; /* GK_READS_* of packed                   */
} gk_host_batch;

int gk_filter_host(gk_ctx *ctx, const gk_host_batch *batch);

/*
 * Verification of filtered pairs: the exact edit distance that a read
 * mapper's verification step computes for the pairs the filter passes
 * (Sec. 3.3, Sec. 3.5): unit-cost global alignment of the read with its
 * window ref[cand_pos[i], cand_pos[i] + m), the ground truth of Sec. 4.4.
 *
 * batch: as for gk_filter (its accept, est and accept_bits are not used).
 * accept: DEVICE, n_pairs codes written by gk_filter / gk_filter_mixed, or
 * NULL to verify every pair.
 * dist: DEVICE out, n_pairs: min(edit distance, e_i + 1) for each pair with
 * accept[i] == GK_ACCEPT (every pair when accept is NULL), so dist <= e_i
 * exactly when the pair lies within e_i edits; GK_EST_NONE for pairs not
 * verified, for pairs gk_filter marks GK_UNDEFINED or GK_INVALID, and for
 * e_i > GK_VERIFY_MAX_E.
 * Asynchronous on stream.  Uses context-owned scratch (two pair lists of up
 * to 2^30 entries each, 8 bytes per pair of the largest batch so far plus a
 * word per 4096 pairs, allocated on first use and grown as needed): calls on
 * one context must not overlap on different streams.  Errors as gk_filter, plus GK_EINVAL for a
 * NULL dist.
 */
#define GK_VERIFY_MAX_E 31u

int gk_verify(gk_ctx *ctx, const gk_batch *batch, const uint8_t *accept, uint16_t *dist,
              void *stream);

/* Tuning options of a context (they never change results). */
#define GK_OPT_PAIRS_PER_LANE 1   /* plain filter grid: 0 (default) =
                                     automatic (currently one pair per
                                     lane); 1 = one pair per lane; k in 2..65535 =
                                     about k pairs per lane, each lane
                                     keeping its next pair's loads in
                                     flight; 65536 = one residency of the
                                     device.  Range 0..65536.                */

#define GK_OPT_MIXED_TILE           2  /* gk_filter_mixed: pairs per tile,
                                            2048, 4096 (default) or 8192    */
#define GK_OPT_MIXED_PAIRS_PER_LANE 3  /* gk_filter_mixed: 1 (default) or 2
                                            pairs per lane per chunk        */
#define GK_OPT_MIXED_SORT_E         4  /* gk_filter_mixed: 1 (default) sorts
                                            a tile by (W, min(e, m-1)), 0 by
                                            W only                          */
#define GK_OPT_MIXED_BLOCKS_PER_CU  5  /* gk_filter_mixed: persistent
                                            workgroups per CU, 0 (default) =
                                            as many as fit, else 1..64      */
#define GK_OPT_MIXED_GRAPH          6  /* gk_filter_mixed: 1 (default)
                                            replays a captured hipGraph, 0
                                            launches directly               */
#define GK_OPT_HOST_ENCODE_THREADS  7  /* gk_filter_host with ASCII reads:
                                            0 (default) copies the text and
                                            encodes it on the GPU; 1..64
                                            encodes it into 2-bit words on
                                            that many host threads, chunk by
                                            chunk while the previous chunk is
                                            copied and filtered, so a quarter
                                            of the bytes cross the bus.  Same
                                            results either way.             */
#define GK_OPT_SERVER_PART_PAIRS    8  /* gk_server_start, batched mode: a
                                            tick takes at most this many
                                            pairs of one request (256..2^30,
                                            default 131072); a larger
                                            request is spread over ticks    */
#define GK_OPT_SERVER_TICK_PAIRS    9  /* gk_server_start, batched mode:
                                            pairs per tick at most
                                            (4096..2^26, default 2^20)      */
#define GK_OPT_HOST_CHUNK_PAIRS    10  /* gk_filter_host: pairs per chunk,
                                            0 (default) = n_pairs / 16
                                            within 2^20..2^22, else 64..2^26
                                            (rounded up to a multiple of
                                            64); sets its device memory     */
#define GK_OPT_SERVER_COPY_STREAMS 11  /* gk_server_start, batched mode:
                                            streams the loader takes in turn
                                            for requests' copies in and
                                            encoding, 1..8 (default 4)      */

/* Set / get a tuning option.  GK_EINVAL for an unknown option or a value out
   of range.  gk_create also takes each option from the environment variable
   GK_<name> of GK_OPT_<name> (GK_MIXED_TILE=8192, GK_HOST_CHUNK_PAIRS=65536,
   ...) when it is set: a value that is not a decimal integer in the option's
   range makes gk_create fail with GK_EINVAL, naming the variable. */
int gk_set_option(gk_ctx *ctx, int option, int64_t value);
int gk_get_option(const gk_ctx *ctx, int option, int64_t *value);

/*
 * Mixed-batch filter: the same per-pair filter as gk_filter for batches whose
 * pairs differ in read length and threshold (the paper compiles both in,
 * Sec. 3.1, and would launch once per (length, e) group).
 *
 * One persistent launch covers the batch: workgroups claim tiles of
 * consecutive pairs from a device counter, counting-sort each tile in LDS by
 * (words per mask, min(e, m-1)) and run each 64-lane chunk through the fast
 * path for its read length; pairs with more than 31 shifts are finished by a
 * general-path pass; accept bits (if requested) by a pass over the accept
 * codes.  The launch sequence is captured in a hipGraph the first time a
 * given shape (words per mask, read layout) and tuning are seen and replayed
 * after that (GK_OPT_MIXED_GRAPH): the batch's arguments reach the graph
 * through a device table that a copy on the stream fills before each replay,
 * so every batch of that shape replays the same graph.  Batches of more than
 * 2^30 pairs, and batches with variant flags, are launched directly.
 * Results are identical to gk_filter's.
 *
 * Same batch rules and errors as gk_filter.  The context keeps scratch for
 * it: two counters, a residual list of min(n_pairs, 2^30) entries (grown on
 * demand), the device argument table and four pinned host copies of it (a
 * call waits until the replay four calls earlier has read its copy), all
 * kept until gk_destroy.  Calls that overlap on one context race on that
 * scratch: one gk_filter_mixed at a time per context, on one stream.
 * Asynchronous on stream.
 */
int gk_filter_mixed(gk_ctx *ctx, const gk_batch *batch, void *stream);

/*
 * gk_filter_mixed for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same batch rules, tuning (GK_OPT_MIXED_*), launch sequence and results as
 * gk_filter_mixed, launched directly on stream (no hipGraph; the graph
 * option is ignored).  It calls no hipMalloc or hipFree and allocates no
 * stream, event or graph.
 *
 * Scratch: the tile counter, the residual count and a residual list of up
 * to GK_NOALLOC_MAX_PAIRS entries live in one fixed device array of the
 * library (16 MiB + 256 B), of which every GPU holds its own copy from the
 * library's load until the process ends; gk_create takes its address on the
 * context's device.  n_pairs above GK_NOALLOC_MAX_PAIRS returns GK_ERANGE
 * with nothing launched; n_pairs == 0 returns GK_OK with nothing launched.
 * Every call on one GPU, from any context and on any stream, uses that GPU's
 * one array, and the array keeps the last call's contents (the launch
 * sequence zeroes the counters first): calls that overlap on one GPU race
 * and give undefined results.  Order them on one stream, or wait for one
 * before starting the next.  Asynchronous on stream.
 */
int gk_filter_mixed_noalloc(gk_ctx *ctx, const gk_batch *batch, void *stream);

/*
 * Autotuner for gk_filter_mixed.  Times every candidate tuning (tile 2048 /
 * 4096 / 8192, 1 or 2 pairs per lane, sort by e or not, full or half
 * persistent grid) on the first sample_pairs pairs of the batch (0 = all),
 * median of 5 runs each after a warm-up, and keeps the fastest in the
 * context.  When it times candidates, the outputs of the sampled pairs are
 * written (correct results: every tuning gives the same ones).  Synchronous.
 *
 * cache_path (HOST string or NULL): a text file of JSON lines keyed by
 * device architecture, CU count, words per mask, read layout, threshold mode
 * and batch size (power-of-two bucket).  The last matching line is used
 * without timing anything; otherwise the measured choice is appended.  A
 * context created with GK_AUTOTUNE=refresh in the environment measures and
 * appends whatever the cache holds; with GK_AUTOTUNE=off it keeps its
 * current tuning, times nothing and reports source "off".
 * report (HOST, report_cap bytes, or NULL): a JSON description of the
 * choice and of every candidate's time, NUL-terminated, truncated to fit.
 */
int gk_tune_mixed(gk_ctx *ctx, const gk_batch *batch, void *stream, uint64_t sample_pairs,
                  const char *cache_path, char *report, size_t report_cap);

/*
 * Serving loop.  Requests of varying size, read length and threshold are
 * submitted from any thread; the server keeps the reference (the context's)
 * and each admitted request's state on the GPU and reports per-request times.
 * The paper has no server: it filters one batch at a time with one
 * synchronisation per batch (Sec. 3.5) and sizes its batches from the
 * device's free memory (Sec. 3.1).  The server generalises both: admission
 * by a device-memory budget, and batches formed from whatever requests are
 * loaded when the device is free (every gk_server_* call below belongs to
 * this addition).
 *
 * GK_SERVER_BATCHED: requests are admitted in arrival order when a slot is
 * free and the device arena (device_budget_bytes, allocated at start) has
 * room for the request's footprint; admitted requests are copied in and
 * encoded on copy streams taken in turn (GK_OPT_SERVER_COPY_STREAMS) while
 * earlier ones are filtered, and every
 * scheduling tick filters parts of the loaded requests together in one
 * persistent launch (the mixed-batch kernel over a table of parts, replayed
 * from a hipGraph), with at most two ticks in flight.  A tick takes the
 * loaded requests in turn, at most GK_OPT_SERVER_PART_PAIRS pairs of each and
 * at most GK_OPT_SERVER_TICK_PAIRS in all; a request with pairs left waits
 * for a later tick behind the others, so a large request does not hold back
 * the small ones loaded after it.  Each part's results are copied back as
 * its tick completes; a request's slot and memory are freed after its last
 * part.  The tick's launch uses the context's mixed-batch tuning
 * (GK_OPT_MIXED_*, e.g. as gk_tune_mixed chose it) and the server options
 * (GK_OPT_SERVER_*) as they are when gk_server_start is called.
 * GK_SERVER_SEQUENTIAL: the per-request baseline: one request at a time, copy
 * in, encode, one plain filter launch, copy out, on one stream.
 * Both give the same bytes as gk_filter on the same pairs.
 */
#define GK_SERVER_BATCHED    0u
#define GK_SERVER_SEQUENTIAL 1u

typedef struct gk_server gk_server;

typedef struct gk_request {
    const char     *reads;         /* HOST: read r = reads[read_off[r] ..
                                      read_off[r+1]), ASCII                 */
    const uint64_t *read_off;      /* HOST: n_reads + 1 offsets              */
    uint32_t        n_reads;       /* < 2^30                                 */
    uint32_t        e;             /* threshold of every pair, 0..255        */
    const uint32_t *pair_read;     /* HOST: n_pairs read indices, or NULL:
                                      pair i uses read i                     */
    const uint32_t *cand_pos;      /* HOST: n_pairs window starts            */
    uint64_t        n_pairs;       /* < 2^30                                 */
    uint8_t        *accept;        /* HOST out: n_pairs result codes         */
    uint16_t       *est;           /* HOST out: n_pairs estimates            */
    int64_t         t_arrival_us;  /* arrival time on gk_clock_us()'s clock
                                      (latency is measured from it), or 0:
                                      the time of submission                 */
} gk_request;

typedef struct gk_request_stats {
    int     status;                /* GK_OK; GK_ECANCELED (stopped before
                                      admission); GK_EDEVICE (server failed) */
    uint64_t n_pairs;
    int64_t t_submit_us;           /* arrival time (t_arrival_us or submit)  */
    int64_t t_admit_us;            /* admitted to a slot                     */
    int64_t t_done_us;             /* results in the caller's host buffers   */
} gk_request_stats;

/* Start a server on ctx's device and resident reference (which must not be
   replaced while the server runs).  max_slots 1..256 requests in flight,
   max_read_len 1..512 (longer requests are refused), device_budget_bytes >=
   1 MiB, mode GK_SERVER_*.  Starts its worker threads. */
int gk_server_start(gk_ctx *ctx, uint64_t device_budget_bytes, uint32_t max_slots,
                    uint32_t max_read_len, uint32_t mode, gk_server **out);

/* Queue a request; returns at once with a ticket.  The host buffers it names
   must stay valid until gk_server_wait returns for the ticket.  GK_EINVAL for
   bad pointers or sizes, GK_ERANGE for reads longer than the server's
   max_read_len or a footprint larger than the whole budget. */
int gk_server_submit(gk_server *srv, const gk_request *req, uint64_t *ticket);

/* Wait for a ticket (timeout_us < 0: no limit).  GK_ETIMEOUT leaves the
   request queued (wait again); any other return releases the ticket.
   Returns the request's status; stats may be NULL.  Thread-safe.
   After a HIP error inside the server, every queued or in-flight request
   ends: GK_OK if its results were already copied out, else GK_EDEVICE.  No
   copy touches its host buffers once its wait has returned.  Later submits
   return GK_EDEVICE, and so does gk_server_stop. */
int gk_server_wait(gk_server *srv, uint64_t ticket, int64_t timeout_us,
                   gk_request_stats *stats);

/* Ticks launched, most request parts in one tick, pairs finished. */
int gk_server_counters(gk_server *srv, uint64_t *ticks, uint64_t *max_requests_per_tick,
                       uint64_t *pairs_done);

/* One scheduling tick of a GK_SERVER_BATCHED server, on gk_clock_us()'s
   clock: when its launch was issued, when the completer saw its kernels
   finish, and when its parts' results were in host memory; n_requests is
   the number of request parts in the tick, n_pairs their pairs. */
typedef struct gk_tick_record {
    int64_t  t_launch_us;
    int64_t  t_kernel_done_us;
    int64_t  t_done_us;
    uint32_t n_requests;
    uint32_t reserved;
    uint64_t n_pairs;
} gk_tick_record;

/* The server's tick log: the first min(cap, n) completed ticks in order are
   copied to out (HOST, cap records; may be NULL when cap is 0), *n_total (may
   be NULL) receives n, the number recorded (the first 2^20 ticks of the
   server are kept).  Empty in GK_SERVER_SEQUENTIAL mode. */
int gk_server_tick_log(gk_server *srv, gk_tick_record *out, uint64_t cap, uint64_t *n_total);

/* Cancel the requests not yet admitted (their status: GK_ECANCELED), finish
   the admitted ones, stop the threads and free the server.  Tickets not yet
   waited for are released. */
int gk_server_stop(gk_server *srv);

/* The clock of gk_request.t_arrival_us and gk_request_stats: microseconds of
   a monotonic clock (CLOCK_MONOTONIC on Linux). */
int64_t gk_clock_us(void);

#ifdef __cplusplus
}
#endif
#endif /* GK_H */

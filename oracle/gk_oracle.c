/*
 * GateKeeper-GPU oracle (TEST INFRASTRUCTURE ONLY; see gk_oracle.h).
 *
 * A deliberately plain restatement of the filter, one base at a time:
 *
 *   Sec. 2.1  2-bit encoding A=00 C=01 G=10 T=11; the Hamming mask is the XOR
 *             of read and window codes with each base's two bits ORed; for
 *             k = 1..e the read is shifted by k bases one way (deletion mask)
 *             and the other way (insertion mask) and compared the same way;
 *             every mask is amended (short 0-streaks become 1s) before the
 *             2e+1 masks are ANDed; the 1s left are counted and the pair is
 *             rejected iff that count exceeds e.
 *   Sec. 3.3  pairs holding a base other than A/C/G/T pass unfiltered.
 *   Sec. 3.4  the shifted masks' vacated leading/trailing bits are set to 1
 *             by one OR after amendment (GateKeeper-GPU's refinement).
 *
 * Readings where the paper is silent or loose (each is also listed in the
 * design notes of the repository):
 *   - a shift by k moves the read by k bases (2k encoded bits);
 *   - positions vacated by a shift compare the window base with code 00
 *     ('A'), as a logical shift of the encoded read fills zeros;
 *   - a "short streak" is a maximal run of one or two 0s with a 1 on both
 *     sides; runs touching either end of the mask are never amended;
 *   - the refinement touches only the k vacated positions of each shifted
 *     mask, after amendment and before the AND; the Hamming mask is never
 *     refined;
 *   - the count is the number of 1s in the final mask;
 *   - e = 0 uses the same steps (only the amended Hamming mask);
 *   - the window is ref[pos, pos+m); a window running past the reference
 *     end is undefined (passed), like a window holding an unknown base.
 */
#include "gk_oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* Sec. 2.1: A = 00, C = 01, G = 10, T = 11.  Lower-case letters are the same
   bases.  Anything else is an unknown base (-1). */
static int base_code(char c)
{
    switch (c) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default:            return -1;
    }
}

int gko_amend(const uint8_t *in, uint32_t m, uint8_t *out)
{
    uint8_t orig[GKO_MAX_LEN];
    uint32_t i, j;
    if (m > GKO_MAX_LEN)
        return -1;
    /* Runs are found on the values before amendment. */
    for (i = 0; i < m; i++)
        orig[i] = in[i];
    for (i = 0; i < m; i++)
        out[i] = orig[i];
    i = 0;
    while (i < m) {
        if (orig[i] != 0) {
            i++;
            continue;
        }
        uint32_t start = i;
        while (i < m && orig[i] == 0)
            i++;
        uint32_t end = i;                 /* run is [start, end) */
        uint32_t len = end - start;
        int bounded_left = start > 0;     /* orig[start-1] == 1 by maximality */
        int bounded_right = end < m;      /* orig[end] == 1 by maximality     */
        if (bounded_left && bounded_right && len <= 2)
            for (j = start; j < end; j++)
                out[j] = 1;
    }
    return 0;
}

/* Mismatch mask for the read shifted by d bases against the window:
   mask[i] = 1 iff code(read[i - d]) differs from code(window[i]); read
   positions outside [0, m) hold code 00.  "Differs" is computed the way the
   paper states it: XOR the two 2-bit codes, then OR the two result bits. */
static void shifted_mask(const int *rc, const int *gc, uint32_t m, int d,
                         uint8_t *mask)
{
    for (uint32_t i = 0; i < m; i++) {
        int j = (int)i - d;
        int r = (j >= 0 && j < (int)m) ? rc[j] : 0;
        int x = r ^ gc[i];
        mask[i] = (uint8_t)(((x >> 1) & 1) | (x & 1));
    }
}

uint32_t gko_filter_pair_trace(const char *read, uint32_t m, const char *ref,
                               uint64_t ref_len, uint64_t pos, uint32_t e,
                               uint32_t flags, uint16_t *est, uint8_t *masks)
{
    int rc[GKO_MAX_LEN], gc[GKO_MAX_LEN];
    uint8_t mask[GKO_MAX_LEN], fin[GKO_MAX_LEN];
    uint32_t i;

    *est = GKO_EST_NONE;
    if (m == 0 || m > GKO_MAX_LEN)
        return GKO_INVALID;
    if (pos > ref_len || ref_len - pos < m)
        return GKO_UNDEFINED;

    /* Encode both sequences; an unknown base makes the pair undefined. */
    for (i = 0; i < m; i++) {
        rc[i] = base_code(read[i]);
        gc[i] = base_code(ref[pos + i]);
        if (rc[i] < 0 || gc[i] < 0)
            return GKO_UNDEFINED;
    }

    /* Optional fast path: accept on the Hamming distance alone. */
    if (flags & GKO_HAMMING_FASTPATH) {
        uint32_t hd = 0;
        for (i = 0; i < m; i++)
            hd += (rc[i] != gc[i]);
        if (hd <= e) {
            *est = (uint16_t)hd;
            return GKO_ACCEPT;
        }
    }

    /* Masks with a shift of m or more bases are all 1s once refined, so
       they never change the AND; stopping at min(e, m) is exact. */
    uint32_t e_eff = e < m ? e : m;

    for (i = 0; i < m; i++)
        fin[i] = 1;

    for (uint32_t slot = 0; slot < 2 * e_eff + 1; slot++) {
        /* slot 0: Hamming mask; slot 2k-1: deletion (+k); slot 2k: insertion (-k). */
        int k = (int)((slot + 1) / 2);
        int d = (slot == 0) ? 0 : ((slot % 2 == 1) ? k : -k);
        uint8_t *rec = masks ? masks + (size_t)slot * 3 * m : NULL;

        shifted_mask(rc, gc, m, d, mask);
        if (rec)
            memcpy(rec + GKO_STAGE_RAW * m, mask, m);

        gko_amend(mask, m, mask);
        if (rec)
            memcpy(rec + GKO_STAGE_AMENDED * m, mask, m);

        if (!(flags & GKO_NO_REFINE)) {
            if (d > 0)                       /* deletion: leading k positions  */
                for (i = 0; i < m && i < (uint32_t)d; i++)
                    mask[i] = 1;
            if (d < 0)                       /* insertion: trailing k positions */
                for (i = 0; i < m; i++)
                    if (i + (uint32_t)(-d) >= m)
                        mask[i] = 1;
        }
        if (rec)
            memcpy(rec + GKO_STAGE_REFINED * m, mask, m);

        for (i = 0; i < m; i++)
            fin[i] = (uint8_t)(fin[i] & mask[i]);
    }

    uint32_t count = 0;
    for (i = 0; i < m; i++)
        count += fin[i];
    *est = (uint16_t)count;
    return count <= e ? GKO_ACCEPT : GKO_REJECT;
}

uint32_t gko_filter_pair(const char *read, uint32_t m, const char *ref,
                         uint64_t ref_len, uint64_t pos, uint32_t e,
                         uint32_t flags, uint16_t *est)
{
    return gko_filter_pair_trace(read, m, ref, ref_len, pos, e, flags, est,
                                 NULL);
}

/* ------------------------------------------------------------------------ */
/* Batch driver: contiguous pair ranges, one POSIX thread per range.         */

typedef struct {
    const char *reads;
    const uint64_t *read_off;
    uint32_t n_reads;
    const char *ref;
    uint64_t ref_len;
    const uint32_t *pair_read;
    const uint32_t *cand_pos;
    const uint8_t *e_pair;
    uint32_t e_uniform;
    uint32_t flags;
    uint32_t cap;
    uint8_t *accept;
    uint16_t *est;
    uint16_t *dist;
    uint64_t begin, end;
} batch_job;

static void *filter_range(void *arg)
{
    batch_job *j = (batch_job *)arg;
    for (uint64_t i = j->begin; i < j->end; i++) {
        uint32_t r = j->pair_read[i];
        uint16_t est = GKO_EST_NONE;
        uint32_t res;
        if (r >= j->n_reads) {
            res = GKO_INVALID;
        } else {
            uint64_t off = j->read_off[r];
            uint64_t len = j->read_off[r + 1] - off;
            uint32_t e = j->e_pair ? j->e_pair[i] : j->e_uniform;
            if (len > GKO_MAX_LEN)
                res = GKO_INVALID;
            else
                res = gko_filter_pair(j->reads + off, (uint32_t)len, j->ref,
                                      j->ref_len, j->cand_pos[i], e, j->flags,
                                      &est);
        }
        j->accept[i] = (uint8_t)res;
        j->est[i] = est;
    }
    return NULL;
}

static void *lev_range(void *arg)
{
    batch_job *j = (batch_job *)arg;
    for (uint64_t i = j->begin; i < j->end; i++) {
        uint32_t r = j->pair_read[i];
        uint32_t d = j->cap + 1;
        if (r < j->n_reads) {
            uint64_t off = j->read_off[r];
            uint64_t len = j->read_off[r + 1] - off;
            uint64_t pos = j->cand_pos[i];
            if (pos <= j->ref_len && j->ref_len - pos >= len)
                d = gko_levenshtein(j->reads + off, (uint32_t)len,
                                    j->ref + pos, (uint32_t)len, j->cap);
        }
        j->dist[i] = (uint16_t)(d > 0xFFFFu ? 0xFFFFu : d);
    }
    return NULL;
}

static int run_threads(batch_job *proto, uint64_t n, uint32_t n_threads,
                       void *(*fn)(void *))
{
    if (n_threads < 1)
        n_threads = 1;
    if (n_threads > 256)
        n_threads = 256;
    if ((uint64_t)n_threads > n)
        n_threads = n > 0 ? (uint32_t)n : 1;
    batch_job jobs[256];
    pthread_t tid[256];
    uint64_t chunk = (n + n_threads - 1) / n_threads;
    for (uint32_t t = 0; t < n_threads; t++) {
        jobs[t] = *proto;
        jobs[t].begin = (uint64_t)t * chunk < n ? (uint64_t)t * chunk : n;
        jobs[t].end = jobs[t].begin + chunk < n ? jobs[t].begin + chunk : n;
    }
    if (n_threads == 1) {
        fn(&jobs[0]);
        return 0;
    }
    uint32_t started = 0;
    for (uint32_t t = 0; t < n_threads; t++) {
        if (pthread_create(&tid[t], NULL, fn, &jobs[t]) != 0)
            break;
        started++;
    }
    for (uint32_t t = started; t < n_threads; t++)
        fn(&jobs[t]);                       /* run what could not be spawned */
    for (uint32_t t = 0; t < started; t++)
        pthread_join(tid[t], NULL);
    return 0;
}

int gko_filter_batch(const char *reads, const uint64_t *read_off,
                     uint32_t n_reads, const char *ref, uint64_t ref_len,
                     const uint32_t *pair_read, const uint32_t *cand_pos,
                     const uint8_t *e_pair, uint32_t e_uniform,
                     uint64_t n_pairs, uint32_t flags, uint32_t n_threads,
                     uint8_t *accept, uint16_t *est)
{
    batch_job p;
    memset(&p, 0, sizeof p);
    p.reads = reads;
    p.read_off = read_off;
    p.n_reads = n_reads;
    p.ref = ref;
    p.ref_len = ref_len;
    p.pair_read = pair_read;
    p.cand_pos = cand_pos;
    p.e_pair = e_pair;
    p.e_uniform = e_uniform;
    p.flags = flags;
    p.accept = accept;
    p.est = est;
    return run_threads(&p, n_pairs, n_threads, filter_range);
}

/* ------------------------------------------------------------------------ */
/* Ground truth: global edit distance with unit costs (the paper uses Edlib's
   global mode for this, Sec. 4.4).                                          */

uint32_t gko_levenshtein_full(const char *a, uint32_t n, const char *b,
                              uint32_t p)
{
    uint32_t *prev = (uint32_t *)malloc(sizeof(uint32_t) * (p + 1));
    uint32_t *cur = (uint32_t *)malloc(sizeof(uint32_t) * (p + 1));
    uint32_t j, i, out;
    if (!prev || !cur) {
        free(prev);
        free(cur);
        return 0xFFFFFFFFu;
    }
    for (j = 0; j <= p; j++)
        prev[j] = j;
    for (i = 1; i <= n; i++) {
        cur[0] = i;
        for (j = 1; j <= p; j++) {
            uint32_t sub = prev[j - 1] + (a[i - 1] != b[j - 1] ? 1u : 0u);
            uint32_t del = prev[j] + 1;
            uint32_t ins = cur[j - 1] + 1;
            uint32_t best = sub < del ? sub : del;
            cur[j] = best < ins ? best : ins;
        }
        uint32_t *t = prev;
        prev = cur;
        cur = t;
    }
    out = prev[p];
    free(prev);
    free(cur);
    return out;
}

uint32_t gko_levenshtein(const char *a, uint32_t n, const char *b, uint32_t p,
                         uint32_t cap)
{
    const uint32_t INF = 0x3FFFFFFFu;
    uint32_t diff = n > p ? n - p : p - n;
    if (diff > cap)
        return cap + 1;
    if (cap >= (n > p ? n : p)) {
        uint32_t d = gko_levenshtein_full(a, n, b, p);
        return d > cap ? cap + 1 : d;
    }
    /* Cells (i, j) with |i - j| > cap cost more than cap, so they are
       treated as infinite; every other cell follows the full recurrence. */
    uint32_t *prev = (uint32_t *)malloc(sizeof(uint32_t) * (p + 1));
    uint32_t *cur = (uint32_t *)malloc(sizeof(uint32_t) * (p + 1));
    uint32_t i, j, out;
    if (!prev || !cur) {
        free(prev);
        free(cur);
        return 0xFFFFFFFFu;
    }
    for (j = 0; j <= p; j++)
        prev[j] = j <= cap ? j : INF;
    for (i = 1; i <= n; i++) {
        uint32_t lo = i > cap ? i - cap : 0;
        uint32_t hi = i + cap < p ? i + cap : p;
        for (j = 0; j <= p; j++)
            cur[j] = INF;
        if (lo == 0)
            cur[0] = i;
        for (j = lo > 1 ? lo : 1; j <= hi; j++) {
            uint32_t sub = prev[j - 1] + (a[i - 1] != b[j - 1] ? 1u : 0u);
            uint32_t del = prev[j] + 1;
            uint32_t ins = cur[j - 1] + 1;
            uint32_t best = sub < del ? sub : del;
            best = best < ins ? best : ins;
            cur[j] = best < INF ? best : INF;
        }
        uint32_t *t = prev;
        prev = cur;
        cur = t;
    }
    out = prev[p];
    free(prev);
    free(cur);
    return out > cap ? cap + 1 : out;
}

int gko_levenshtein_batch(const char *reads, const uint64_t *read_off,
                          uint32_t n_reads, const char *ref, uint64_t ref_len,
                          const uint32_t *pair_read, const uint32_t *cand_pos,
                          uint64_t n_pairs, uint32_t cap, uint32_t n_threads,
                          uint16_t *dist)
{
    batch_job p;
    memset(&p, 0, sizeof p);
    p.reads = reads;
    p.read_off = read_off;
    p.n_reads = n_reads;
    p.ref = ref;
    p.ref_len = ref_len;
    p.pair_read = pair_read;
    p.cand_pos = cand_pos;
    p.cap = cap;
    p.dist = dist;
    return run_threads(&p, n_pairs, n_threads, lev_range);
}

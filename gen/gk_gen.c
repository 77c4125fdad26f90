/*
 * Seeded synthetic workloads for the GateKeeper filter: references, reads
 * with edits, candidate positions and thresholds.  Used by both the tests
 * (oracle side and HIP side) and the benchmark.  It holds none of the
 * filter's arithmetic: no encoding, no masks, no counting; it only writes
 * ASCII sequences and integer positions.
 *
 * Randomness: every read (and every reference block) draws from its own
 * SplitMix64 stream keyed by (seed, stream id, index), so the output does
 * not depend on the number of threads.
 *
 * The paper measured 100/150/250 bp reads paired with candidate positions
 * produced by mrFAST, Minimap2 and BWA-MEM seeding on real data (Sec. 4.1);
 * those sets are not available, so these generators stand in with the same
 * shapes: read lengths, thresholds up to 10% of the read length, true
 * origins with sequencing-like edits, and seed-sharing decoys.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- RNG --- */

typedef struct { uint64_t s; } rng_t;

static uint64_t splitmix_next(rng_t *r)
{
    uint64_t z = (r->s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static rng_t rng_for(uint64_t seed, uint64_t stream, uint64_t index)
{
    rng_t r;
    r.s = seed * 0xD1B54A32D192ED03ull ^ stream * 0xABC98388FB8FAC03ull ^
          index * 0x8CB92BA72F3D8DD7ull;
    splitmix_next(&r);
    splitmix_next(&r);
    return r;
}

/* Uniform double in [0, 1). */
static double rng_unit(rng_t *r) { return (splitmix_next(r) >> 11) * (1.0 / 9007199254740992.0); }

/* Uniform integer in [0, n). */
static uint64_t rng_below(rng_t *r, uint64_t n)
{
    if (n <= 1)
        return 0;
    return (uint64_t)(rng_unit(r) * (double)n) % n;
}

static uint32_t rng_poisson(rng_t *r, double lambda)
{
    if (lambda <= 0)
        return 0;
    if (lambda > 60) {                       /* normal approximation */
        double u1 = rng_unit(r) + 1e-300, u2 = rng_unit(r);
        double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
        double v = lambda + z * sqrt(lambda) + 0.5;
        return v < 0 ? 0 : (uint32_t)v;
    }
    double L = exp(-lambda), p = 1.0;
    uint32_t k = 0;
    do {
        k++;
        p *= rng_unit(r);
    } while (p > L);
    return k - 1;
}

static uint32_t rng_binomial(rng_t *r, uint32_t n, double p)
{
    uint32_t k = 0;
    for (uint32_t i = 0; i < n; i++)
        k += rng_unit(r) < p;
    return k;
}

/* Geometric on {1, 2, ...} with success probability p, capped. */
static uint32_t rng_geometric(rng_t *r, double p, uint32_t cap)
{
    uint32_t c = 1;
    while (c < cap && rng_unit(r) >= p)
        c++;
    return c;
}

/* Zipf(s) on {1..cap} by inversion of the precomputed CDF. */
static uint32_t rng_zipf(rng_t *r, const double *cdf, uint32_t cap)
{
    double u = rng_unit(r);
    uint32_t lo = 0, hi = cap - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi) / 2;
        if (cdf[mid] < u)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo + 1;
}

static const char BASES[4] = {'A', 'C', 'G', 'T'};

/* Base with P(C) = P(G) = gc/2, P(A) = P(T) = (1-gc)/2. */
static char rng_base(rng_t *r, double gc)
{
    double u = rng_unit(r);
    double at = (1.0 - gc) / 2, g = gc / 2;
    if (u < at) return 'A';
    if (u < at + g) return 'C';
    if (u < at + 2 * g) return 'G';
    return 'T';
}

/* ---------------------------------------------------------- reference --- */

typedef struct {
    uint8_t *out;
    uint64_t len, begin, end;
    double gc;
    uint64_t seed;
} ref_job;

#define REF_BLOCK 65536u

static void *ref_range(void *arg)
{
    ref_job *j = (ref_job *)arg;
    for (uint64_t b = j->begin; b < j->end; b++) {
        rng_t r = rng_for(j->seed, 1, b);
        uint64_t lo = b * REF_BLOCK, hi = lo + REF_BLOCK < j->len ? lo + REF_BLOCK : j->len;
        for (uint64_t i = lo; i < hi; i++)
            j->out[i] = (uint8_t)rng_base(&r, j->gc);
    }
    return NULL;
}

static uint32_t clamp_threads(uint32_t t)
{
    return t < 1 ? 1 : (t > 64 ? 64 : t);
}

/* i.i.d. reference of len bases with GC fraction gc (0.5 = uniform). */
int gkg_reference(uint8_t *out, uint64_t len, double gc, uint64_t seed, uint32_t n_threads)
{
    n_threads = clamp_threads(n_threads);
    uint64_t nb = (len + REF_BLOCK - 1) / REF_BLOCK;
    ref_job jobs[64];
    pthread_t tid[64];
    uint64_t chunk = (nb + n_threads - 1) / n_threads;
    for (uint32_t t = 0; t < n_threads; t++) {
        jobs[t].out = out;
        jobs[t].len = len;
        jobs[t].gc = gc;
        jobs[t].seed = seed;
        jobs[t].begin = t * chunk < nb ? t * chunk : nb;
        jobs[t].end = jobs[t].begin + chunk < nb ? jobs[t].begin + chunk : nb;
        pthread_create(&tid[t], NULL, ref_range, &jobs[t]);
    }
    for (uint32_t t = 0; t < n_threads; t++)
        pthread_join(tid[t], NULL);
    return 0;
}

/* --------------------------------------------------------------- pairs --- */

/* Pair classes reported with each pair. */
enum { CLS_ORIGIN = 0, CLS_BAND = 1, CLS_SEEDED = 2, CLS_RANDOM = 3 };

/* Candidate-count distributions. */
enum { CAND_ONE = 0, CAND_GEOM = 1, CAND_ZIPF = 2 };
/* Edit models for true reads. */
enum { EDIT_POISSON = 0, EDIT_RATE = 1 };
/* Decoy models. */
enum { DECOY_RANDOM_POS = 0, DECOY_SPLICE_KMER = 1, DECOY_SEEDS = 2 };

typedef struct {
    uint64_t seed;
    uint32_t n_reads;
    const uint16_t *len_choices;  /* read length drawn uniformly from these */
    uint32_t n_len_choices;
    int cand_kind;                /* CAND_* */
    double cand_param;            /* geometric p, or Zipf exponent s */
    uint32_t cand_cap;
    double true_frac;             /* fraction of reads built from an origin */
    int edit_kind;                /* EDIT_* */
    double edit_param;            /* Poisson lambda, or rate factor f: rho ~ U[0, f*e/m] */
    int decoy_kind;               /* DECOY_* */
    uint32_t seed_k;              /* k-mer length for spliced / seeded decoys */
    int e_kind;                   /* 0: e_value for all; 1: per pair U{0..floor(e_frac*m)} */
    uint32_t e_value;
    double e_frac;
    double gc;                    /* composition of decoy read bodies */
    int band_cands;               /* true reads: extra candidates at origin +- delta, |delta| <= e */
    uint32_t n_true_first;        /* if nonzero: reads [0, n) are true, the rest decoys */
} gkg_params;

typedef struct {
    const gkg_params *p;
    const uint8_t *ref;
    uint64_t ref_len;
    const double *zipf_cdf;
    /* outputs */
    uint16_t *read_len;            /* per read */
    uint32_t *n_cand;              /* per read */
    uint64_t *read_off;            /* per read + 1 (pass 2) */
    uint64_t *pair_off;            /* per read + 1 (pass 2) */
    uint8_t *reads;
    uint32_t *pair_read, *cand_pos;
    uint8_t *pair_e, *pair_cls;
    uint32_t begin, end;
    int pass;
} pair_job;

static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

static uint32_t e_for(const gkg_params *p, rng_t *r, uint32_t m)
{
    if (p->e_kind == 0)
        return p->e_value;
    uint32_t emax = (uint32_t)floor(p->e_frac * m + 1e-9);
    return (uint32_t)rng_below(r, (uint64_t)emax + 1);
}

/* Read of length m taken from ref at origin o with k edits applied right to
   left at uniform positions in [0, m): substitution 70% (a different base),
   insertion 15% (1-3 random bases), deletion 15% (1-3 bases).  The first m
   bases of the result are kept. */
static void edited_read(rng_t *r, const uint8_t *ref, uint64_t o, uint32_t m, uint32_t k,
                        char *out, char *work, uint32_t work_cap)
{
    uint32_t len = m + 3 * k;
    if (len > work_cap)
        len = work_cap;
    memcpy(work, ref + o, len);
    uint32_t pos[1024];
    uint32_t nk = k < 1024 ? k : 1024;
    for (uint32_t i = 0; i < nk; i++)
        pos[i] = (uint32_t)rng_below(r, m);
    /* sort descending (insertion sort; nk is small) */
    for (uint32_t i = 1; i < nk; i++) {
        uint32_t v = pos[i], j = i;
        while (j > 0 && pos[j - 1] < v) {
            pos[j] = pos[j - 1];
            j--;
        }
        pos[j] = v;
    }
    for (uint32_t i = 0; i < nk; i++) {
        uint32_t x = pos[i];
        double u = rng_unit(r);
        if (x >= len)
            continue;
        if (u < 0.70) {
            char c = work[x], n;
            do {
                n = BASES[rng_below(r, 4)];
            } while (n == c);
            work[x] = n;
        } else if (u < 0.85) {
            uint32_t L = 1 + (uint32_t)rng_below(r, 3);
            if (len + L > work_cap)
                L = work_cap - len;
            memmove(work + x + L, work + x, len - x);
            for (uint32_t t = 0; t < L; t++)
                work[x + t] = BASES[rng_below(r, 4)];
            len += L;
        } else {
            uint32_t L = 1 + (uint32_t)rng_below(r, 3);
            if (x + L > len)
                L = len - x;
            memmove(work + x, work + x + L, len - x - L);
            len -= L;
        }
    }
    /* Deletions can shorten below m: extend with the reference that follows. */
    uint32_t have = len < m ? len : m;
    memcpy(out, work, have);
    for (uint32_t i = have; i < m; i++)
        out[i] = BASES[rng_below(r, 4)];
}

static uint32_t cand_count(const gkg_params *p, rng_t *r, const double *zcdf)
{
    switch (p->cand_kind) {
    case CAND_GEOM: return rng_geometric(r, p->cand_param, p->cand_cap);
    case CAND_ZIPF: return rng_zipf(r, zcdf, p->cand_cap);
    default: return 1;
    }
}

/* Pass 1 draws only what sizes the output (length, candidate count), from a
   stream separate from the one that fills the read, so pass 2 can repeat it. */
static void *pairs_range(void *arg)
{
    pair_job *j = (pair_job *)arg;
    const gkg_params *p = j->p;
    char work[4096];
    for (uint32_t ri = j->begin; ri < j->end; ri++) {
        rng_t rs = rng_for(p->seed, 2, ri);
        uint32_t m = p->len_choices[rng_below(&rs, p->n_len_choices)];
        uint32_t c = cand_count(p, &rs, j->zipf_cdf);
        if (j->pass == 1) {
            j->read_len[ri] = (uint16_t)m;
            j->n_cand[ri] = c;
            continue;
        }
        rng_t r = rng_for(p->seed, 3, ri);
        char *rd = (char *)j->reads + j->read_off[ri];
        uint64_t base = j->pair_off[ri];
        uint64_t span = j->ref_len > m + 16 ? j->ref_len - m - 16 : 1;
        double u_true = rng_unit(&r);
        int is_true = p->n_true_first ? ri < p->n_true_first : u_true < p->true_frac;
        /* e drawn per pair; the first pair's e also sets the read's edit rate */
        uint32_t es[1024];
        for (uint32_t t = 0; t < c && t < 1024; t++)
            es[t] = e_for(p, &r, m);
        uint32_t e_read = es[0];
        for (uint32_t t = 1; t < c && t < 1024; t++)
            if (es[t] > e_read)
                e_read = es[t];
        if (is_true) {
            uint32_t k;
            if (p->edit_kind == EDIT_POISSON)
                k = rng_poisson(&r, p->edit_param);
            else {
                double rho = rng_unit(&r) * p->edit_param * (double)e_read / (double)m;
                k = rng_binomial(&r, m, clampd(rho, 0, 1));
            }
            if (k > 300)
                k = 300;
            uint64_t room = j->ref_len > m + 3ull * k + 1 ? j->ref_len - m - 3ull * k - 1 : 1;
            uint64_t o = rng_below(&r, room);
            edited_read(&r, j->ref, o, m, k, rd, work, sizeof work);
            /* candidates: origin, then distinct band shifts, then random */
            uint32_t used = 0;
            j->cand_pos[base] = (uint32_t)o;
            j->pair_cls[base] = CLS_ORIGIN;
            used = 1;
            if (p->band_cands) {
                uint32_t band = e_read;
                int32_t deltas[64];
                uint32_t nd = 0;
                for (uint32_t dd = 1; dd <= band && nd + 2 <= 64; dd++) {
                    deltas[nd++] = (int32_t)dd;
                    deltas[nd++] = -(int32_t)dd;
                }
                /* shuffle the band shifts */
                for (uint32_t t = nd; t > 1; t--) {
                    uint32_t s = (uint32_t)rng_below(&r, t);
                    int32_t tmp = deltas[t - 1];
                    deltas[t - 1] = deltas[s];
                    deltas[s] = tmp;
                }
                for (uint32_t t = 0; t < nd && used < c; t++) {
                    int64_t q = (int64_t)o + deltas[t];
                    if (q < 0 || (uint64_t)q + m > j->ref_len)
                        continue;
                    j->cand_pos[base + used] = (uint32_t)q;
                    j->pair_cls[base + used] = CLS_BAND;
                    used++;
                }
            }
            for (; used < c; used++) {
                j->cand_pos[base + used] = (uint32_t)rng_below(&r, span);
                j->pair_cls[base + used] = CLS_RANDOM;
            }
        } else {
            if (p->decoy_kind == DECOY_RANDOM_POS) {
                /* An edited read from some origin, paired with unrelated positions. */
                uint32_t k = p->edit_kind == EDIT_POISSON ? rng_poisson(&r, p->edit_param) : 0;
                if (k > 300)
                    k = 300;
                uint64_t room = j->ref_len > m + 3ull * k + 1 ? j->ref_len - m - 3ull * k - 1 : 1;
                uint64_t o = rng_below(&r, room);
                edited_read(&r, j->ref, o, m, k, rd, work, sizeof work);
                for (uint32_t t = 0; t < c; t++) {
                    j->cand_pos[base + t] = (uint32_t)rng_below(&r, span);
                    j->pair_cls[base + t] = CLS_RANDOM;
                }
            } else if (p->decoy_kind == DECOY_SPLICE_KMER) {
                /* A genome-like read from an unrelated origin with the exact
                   k-mer ref[q+o, q+o+K) spliced in at offset o; paired with q. */
                uint32_t K = p->seed_k < m ? p->seed_k : m;
                uint64_t o2 = rng_below(&r, span);
                memcpy(rd, j->ref + o2, m);
                for (uint32_t t = 0; t < c; t++) {
                    uint64_t q = rng_below(&r, span);
                    uint32_t off = (uint32_t)rng_below(&r, m - K + 1);
                    if (t == 0)
                        memcpy(rd + off, j->ref + q + off, K);
                    j->cand_pos[base + t] = (uint32_t)q;
                    j->pair_cls[base + t] = t == 0 ? CLS_SEEDED : CLS_RANDOM;
                }
            } else {
                /* Random read body carrying up to floor(m/K) non-overlapping
                   exact K-mers, each copied from its own reference site; the
                   candidate of a seed is its site minus its offset. */
                uint32_t K = p->seed_k < m ? p->seed_k : m;
                for (uint32_t t = 0; t < m; t++)
                    rd[t] = rng_base(&r, p->gc);
                uint32_t slots = m / K;
                uint32_t ns = c < slots ? c : slots;
                for (uint32_t t = 0; t < c; t++) {
                    if (t < ns) {
                        uint32_t off = t * K;
                        uint64_t site = off + rng_below(&r, span > off ? span - off : 1);
                        if (site + K > j->ref_len)
                            site = off;
                        memcpy(rd + off, j->ref + site, K);
                        j->cand_pos[base + t] = (uint32_t)(site - off);
                        j->pair_cls[base + t] = CLS_SEEDED;
                    } else {
                        j->cand_pos[base + t] = (uint32_t)rng_below(&r, span);
                        j->pair_cls[base + t] = CLS_RANDOM;
                    }
                }
            }
        }
        for (uint32_t t = 0; t < c; t++) {
            j->pair_read[base + t] = ri;
            j->pair_e[base + t] = (uint8_t)(t < 1024 ? es[t] : es[0]);
        }
    }
    return NULL;
}

static void run_pairs(pair_job *proto, uint32_t n_reads, uint32_t n_threads)
{
    n_threads = clamp_threads(n_threads);
    pair_job jobs[64];
    pthread_t tid[64];
    uint32_t chunk = (n_reads + n_threads - 1) / n_threads;
    for (uint32_t t = 0; t < n_threads; t++) {
        jobs[t] = *proto;
        jobs[t].begin = t * chunk < n_reads ? t * chunk : n_reads;
        jobs[t].end = jobs[t].begin + chunk < n_reads ? jobs[t].begin + chunk : n_reads;
        pthread_create(&tid[t], NULL, pairs_range, &jobs[t]);
    }
    for (uint32_t t = 0; t < n_threads; t++)
        pthread_join(tid[t], NULL);
}

static double *zipf_table(const gkg_params *p)
{
    if (p->cand_kind != CAND_ZIPF)
        return NULL;
    double *cdf = (double *)malloc(sizeof(double) * p->cand_cap);
    double s = 0;
    for (uint32_t c = 1; c <= p->cand_cap; c++)
        s += pow((double)c, -p->cand_param);
    double acc = 0;
    for (uint32_t c = 1; c <= p->cand_cap; c++) {
        acc += pow((double)c, -p->cand_param) / s;
        cdf[c - 1] = acc;
    }
    cdf[p->cand_cap - 1] = 1.0;
    return cdf;
}

/* Pass 1: per-read lengths and candidate counts (sizes the buffers). */
int gkg_pairs_sizes(const gkg_params *p, uint16_t *read_len, uint32_t *n_cand, uint32_t n_threads)
{
    pair_job j;
    memset(&j, 0, sizeof j);
    j.p = p;
    double *z = zipf_table(p);
    j.zipf_cdf = z;
    j.read_len = read_len;
    j.n_cand = n_cand;
    j.pass = 1;
    run_pairs(&j, p->n_reads, n_threads);
    free(z);
    return 0;
}

/* Pass 2: fill reads (ASCII at read_off), pairs (pair_read, cand_pos, e, class). */
int gkg_pairs_fill(const gkg_params *p, const uint8_t *ref, uint64_t ref_len,
                   const uint64_t *read_off, const uint64_t *pair_off, uint8_t *reads,
                   uint32_t *pair_read, uint32_t *cand_pos, uint8_t *pair_e,
                   uint8_t *pair_cls, uint32_t n_threads)
{
    pair_job j;
    memset(&j, 0, sizeof j);
    j.p = p;
    double *z = zipf_table(p);
    j.zipf_cdf = z;
    j.ref = ref;
    j.ref_len = ref_len;
    j.read_off = (uint64_t *)read_off;
    j.pair_off = (uint64_t *)pair_off;
    j.reads = reads;
    j.pair_read = pair_read;
    j.cand_pos = cand_pos;
    j.pair_e = pair_e;
    j.pair_cls = pair_cls;
    j.pass = 2;
    run_pairs(&j, p->n_reads, n_threads);
    free(z);
    return 0;
}

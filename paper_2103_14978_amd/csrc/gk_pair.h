// Per-pair GateKeeper-GPU filter body for gfx950, shared by the plain and the
// mixed-batch kernels.
//
// One lane filters one (read, candidate) pair, as the paper gives one thread
// to one filtration (Sec. 3.2).  Unlike the paper's kernel, which keeps 2e+1
// masks of 2-bit-interleaved words in thread-local stack arrays, the lane:
//   - holds the read and the window as two bit-planes (high and low code bit)
//     of 32 bases per 32-bit register, so "XOR the codes, OR the two bits"
//     (Sec. 2.1) is (rh ^ gh) | (rl ^ gl) over 32 bases;
//   - gathers the window from the resident bit-plane reference with funnel
//     shifts (v_alignbit) at any base offset;
//   - never stores a mask: each of the 2e+1 masks is built, amended, refined
//     and ANDed into one running accumulator of W registers;
//   - amends with neighbour funnels and 3-input logic (v_bitop3) instead of a
//     look-up table, and counts with v_bcnt instead of a table.
//
// Steps per pair, all from Sec. 2.1 unless noted:
//   H        = mismatch(read, window)
//   D_k, I_k = mismatch(read shifted by +k / -k bases, window), k = 1..e;
//              vacated read positions hold code 00 (a logical shift)
//   each mask is amended: a 0-run of length 1 or 2 with a 1 on both sides
//              inside [0, m) becomes 1s (runs touching either end stay)
//   refinement (Sec. 3.4): after amendment D_k[0, k) and I_k[m-k, m) := 1
//   F        = H & AND_k (D_k & I_k);  est = popcount(F);  accept iff est <= e
// Masks with k >= m are all 1s after refinement, so k stops at min(e, m-1).
// Pairs whose read or window holds an unknown base, or whose window runs past
// the reference end, are passed as GK_UNDEFINED (Sec. 3.3).
#pragma once

#include "gk_args.h"

namespace gkd {

__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t s)
{
    // ({hi, lo} >> s)[31:0] for s in [0, 31]
    return __builtin_amdgcn_alignbit(hi, lo, s);
}

__device__ __forceinline__ uint32_t ones_below(int n)
{
    // bits [0, n) set, n clamped to [0, 32]
    n = n < 0 ? 0 : (n > 32 ? 32 : n);
    return n >= 32 ? 0xFFFFFFFFu : ((1u << n) - 1u);
}

// Three delta swaps on 16 interleaved 2-bit codes (base j in bits 2j, 2j+1):
// afterwards byte 0 holds the low code bits of bases 0-7, byte 1 their high
// bits, byte 2 the low bits of bases 8-15 and byte 3 their high bits.
__device__ __forceinline__ uint32_t unzip3(uint32_t x)
{
    uint32_t t;
    t = (x ^ (x >> 1)) & 0x22222222u; x = x ^ t ^ (t << 1);
    t = (x ^ (x >> 2)) & 0x0C0C0C0Cu; x = x ^ t ^ (t << 2);
    t = (x ^ (x >> 4)) & 0x00F000F0u; x = x ^ t ^ (t << 4);
    return x;
}

// Two read words (bases 0-15 and 16-31 of a 32-base group) -> bit-planes.
template <int L>
__device__ __forceinline__ void planes_from_words(uint32_t p0, uint32_t p1, uint32_t &hi,
                                                  uint32_t &lo)
{
    if (L == GK_READS_SPLIT) {
        // low code bits in bits 0-15, high code bits in bits 16-31
        lo = __builtin_amdgcn_perm(p1, p0, 0x05040100u);
        hi = __builtin_amdgcn_perm(p1, p0, 0x07060302u);
    } else {
        const uint32_t x0 = unzip3(p0), x1 = unzip3(p1);
        lo = __builtin_amdgcn_perm(x1, x0, 0x06040200u);
        hi = __builtin_amdgcn_perm(x1, x0, 0x07050301u);
    }
}

// Amend mask M (W words, bits at or beyond m are 0) and AND (A | X) into acc.
// A 0 at position i is amended iff it lies in a 0-run of length 1 or 2 with
// 1s on both sides: M[i-1]&M[i+1] | M[i-1]&M[i+2] | M[i-2]&M[i+1].
// Positions outside [0, m) read as 0, so runs touching an end never qualify.
template <int W>
__device__ __forceinline__ void amend_and(const uint32_t (&M)[W], uint32_t (&acc)[W],
                                          const uint32_t (&X)[W])
{
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const uint32_t prev = w > 0 ? M[w - 1] : 0u;
        const uint32_t next = w < W - 1 ? M[w + 1] : 0u;
        const uint32_t l1 = funnel(M[w], prev, 31);   // M[i-1]
        const uint32_t l2 = funnel(M[w], prev, 30);   // M[i-2]
        const uint32_t r1 = funnel(next, M[w], 1);    // M[i+1]
        const uint32_t r2 = funnel(next, M[w], 2);    // M[i+2]
        const uint32_t amended = M[w] | (l1 & (r1 | r2)) | (l2 & r1);
        acc[w] &= amended | X[w];
    }
}

template <int W>
__device__ __forceinline__ void mismatch(const uint32_t (&sh)[W], const uint32_t (&sl)[W],
                                         const uint32_t (&gh)[W], const uint32_t (&gl)[W],
                                         uint32_t (&M)[W])
{
#pragma unroll
    for (int w = 0; w < W; ++w)
        M[w] = (sh[w] ^ gh[w]) | (sl[w] ^ gl[w]);
}

// Fast path: every word but the top one is fully inside the read
// (32(W-1) < m <= 32W) and k <= 31, so the refined positions of D_k lie in
// word 0 and those of I_k in words W-2 and W-1.  Read and window planes have
// no bits at or beyond m.
template <int W, bool REFINE = true>
__device__ __forceinline__ uint32_t filter_exact(const uint32_t (&rh)[W], const uint32_t (&rl)[W],
                                                 const uint32_t (&gh)[W], const uint32_t (&gl)[W],
                                                 uint32_t m, uint32_t kmax)
{
    const uint32_t vtop = ones_below((int)m - 32 * (W - 1));  // valid bits of the top word
    uint32_t acc[W], M[W], X[W], sh[W], sl[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        acc[w] = 0xFFFFFFFFu;
        X[w] = 0u;
    }
    mismatch<W>(rh, rl, gh, gl, M);            // Hamming mask (never refined)
    amend_and<W>(M, acc, X);

    // Deletion masks: read[i-k] against window[i]; refined on [0, k).
    uint32_t lead = 0u;
    for (uint32_t k = 1; k <= kmax; ++k) {
        lead = (lead << 1) | 1u;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            sh[w] = w > 0 ? funnel(rh[w], rh[w - 1], 32u - k) : (rh[0] << k);
            sl[w] = w > 0 ? funnel(rl[w], rl[w - 1], 32u - k) : (rl[0] << k);
        }
        mismatch<W>(sh, sl, gh, gl, M);
        M[W - 1] &= vtop;                      // bases moved past the read end
        uint32_t Xd[W];
#pragma unroll
        for (int w = 0; w < W; ++w)
            Xd[w] = (REFINE && w == 0) ? lead : 0u;
        amend_and<W>(M, acc, Xd);
    }

    // Insertion masks: read[i+k] against window[i]; refined on [m-k, m).
    for (uint32_t k = 1; k <= kmax; ++k) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
            sh[w] = w < W - 1 ? funnel(rh[w + 1], rh[w], k) : (rh[W - 1] >> k);
            sl[w] = w < W - 1 ? funnel(rl[w + 1], rl[w], k) : (rl[W - 1] >> k);
        }
        mismatch<W>(sh, sl, gh, gl, M);
        // With V = valid bits of words (W-2, W-1) = (all ones, vtop), the
        // positions >= m-k are those where (V >> k) is 0.  Bits at or above m
        // may be set in Xi: acc is already 0 there.
        uint32_t Xi[W];
#pragma unroll
        for (int w = 0; w < W; ++w)
            Xi[w] = 0u;
        if (REFINE) {
            Xi[W - 1] = ~(vtop >> k);
            if (W >= 2)
                Xi[W >= 2 ? W - 2 : 0] = ~funnel(vtop, 0xFFFFFFFFu, k);
        }
        amend_and<W>(M, acc, Xi);
    }

    uint32_t est = 0;
#pragma unroll
    for (int w = 0; w < W; ++w)
        est += __builtin_popcount(acc[w]);
    return est;
}

// Read r's plane words 0..W-1 from global memory (words at or beyond the read
// length are 0), for the general path.
template <int W, int L>
__device__ __forceinline__ void load_read(const FilterArgs &a, uint32_t r, uint32_t m,
                                          uint32_t (&rh)[W], uint32_t (&rl)[W])
{
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const uint32_t *row0 = a.reads + (size_t)(2 * w) * a.pitch;
        const uint32_t *row1 = a.reads + (size_t)(2 * w + 1) * a.pitch;
        const uint32_t p0 = (m > 32u * w) ? row0[r] : 0u;
        const uint32_t p1 = (m > 32u * w + 16u) ? row1[r] : 0u;
        planes_from_words<L>(p0, p1, rh[w], rl[w]);
    }
}

// General path: any m <= 32W and any k <= m-1 <= 511.  Shifts of 32 bases or
// more move whole words: the read planes are shifted in place by one word each
// time k passes a multiple of 32, and rebuilt between the deletion and the
// insertion loop: reloaded from the read rows in memory, or, with KEPT (reads
// that exist only in registers), taken again from the pair's words.
template <int W, int L, bool REFINE = true, bool KEPT = false>
__device__ __forceinline__ uint32_t filter_general(const FilterArgs &a, uint32_t r,
                                                   const uint32_t (&words)[2 * W],
                                                   uint32_t (&rh)[W], uint32_t (&rl)[W],
                                                   const uint32_t (&gh)[W],
                                                   const uint32_t (&gl)[W], uint32_t m,
                                                   uint32_t kmax)
{
    uint32_t V[W], acc[W], M[W], X[W], sh[W], sl[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        V[w] = ones_below((int)m - 32 * w);
        rh[w] &= V[w];
        rl[w] &= V[w];
        acc[w] = 0xFFFFFFFFu;
        X[w] = 0u;
    }
    mismatch<W>(rh, rl, gh, gl, M);
    amend_and<W>(M, acc, X);

    for (uint32_t k = 1; k <= kmax; ++k) {
        if (k > 1 && ((k - 1) & 31u) == 0u) {  // read moves up one more word
#pragma unroll
            for (int w = W - 1; w >= 0; --w) {
                rh[w] = w > 0 ? rh[w - 1] : 0u;
                rl[w] = w > 0 ? rl[w - 1] : 0u;
            }
        }
        const uint32_t s = 32u - (k - ((k - 1) & ~31u));  // in [0, 31]
#pragma unroll
        for (int w = 0; w < W; ++w) {
            sh[w] = funnel(rh[w], w > 0 ? rh[w - 1] : 0u, s);
            sl[w] = funnel(rl[w], w > 0 ? rl[w - 1] : 0u, s);
        }
        mismatch<W>(sh, sl, gh, gl, M);
#pragma unroll
        for (int w = 0; w < W; ++w) {
            M[w] &= V[w];
            X[w] = REFINE ? ones_below((int)k - 32 * w) : 0u;
        }
        amend_and<W>(M, acc, X);
    }

    if constexpr (KEPT) {
#pragma unroll
        for (int w = 0; w < W; ++w)
            planes_from_words<L>(words[2 * w], words[2 * w + 1], rh[w], rl[w]);
    } else {
        load_read<W, L>(a, r, m, rh, rl);
    }
#pragma unroll
    for (int w = 0; w < W; ++w) {
        rh[w] &= V[w];
        rl[w] &= V[w];
    }
    for (uint32_t k = 1; k <= kmax; ++k) {
        if ((k & 31u) == 0u) {                 // read moves down one more word
#pragma unroll
            for (int w = 0; w < W; ++w) {
                rh[w] = w < W - 1 ? rh[w + 1] : 0u;
                rl[w] = w < W - 1 ? rl[w + 1] : 0u;
            }
        }
        const uint32_t s = k & 31u;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            sh[w] = funnel(w < W - 1 ? rh[w + 1] : 0u, rh[w], s);
            sl[w] = funnel(w < W - 1 ? rl[w + 1] : 0u, rl[w], s);
        }
        mismatch<W>(sh, sl, gh, gl, M);
#pragma unroll
        for (int w = 0; w < W; ++w)
            X[w] = REFINE ? V[w] & ~ones_below((int)m - (int)k - 32 * w) : 0u;
        amend_and<W>(M, acc, X);
    }

    uint32_t est = 0;
#pragma unroll
    for (int w = 0; w < W; ++w)
        est += __builtin_popcount(acc[w]);
    return est;
}

// Indices of one pair (first-level loads).
struct PairIdx {
    uint32_t r, pos, e;
};

// Second-level loads of one pair: read length, read words, window words.
// Issued speculatively (indices clamped into range) so that they can be in
// flight before the pair's validity is known.
template <int W>
struct PairData {
    uint32_t m;
    uint32_t words[2 * W];
    uint2 win[W + 1];
};

// Loads of data that is used once (a.stream_reads: one pair per read, each
// pair entry read once) are non-temporal, so that the L2 keeps the reference
// lines; shared reads (several candidates per read) stay cached.
template <typename T>
__device__ __forceinline__ T ld_once(const FilterArgs &a, const T *p)
{
    return a.stream_reads ? __builtin_nontemporal_load(p) : *p;
}

__device__ __forceinline__ PairIdx load_idx(const FilterArgs &a, uint32_t i)
{
    PairIdx p;
    p.r = a.pair_read ? ld_once(a, a.pair_read + i) : i;
    p.pos = ld_once(a, a.cand_pos + i);
    p.e = a.e_pair ? (uint32_t)ld_once(a, a.e_pair + i) : a.e_uniform;
    return p;
}

// The window words of a pair: only those a window of up to max_read_len
// bases can touch, from the copy of the planes in which they share one
// 128-byte line.
template <int W>
__device__ __forceinline__ void load_window(const FilterArgs &a, uint32_t pos, PairData<W> &d)
{
    pos = pos < a.ref_len ? pos : 0u;
    const uint32_t w0 = pos >> 5;
    const uint32_t span = (pos & 31u) + a.max_read_len;
    const uint32_t nw = (span + 31u) >> 5;
    const bool use_b = a.ref_planes_b != nullptr && w0 >= REF_SHIFT_WORDS &&
                       (w0 & (LINE_WORDS - 1u)) + nw > LINE_WORDS;
    const uint2 *src = use_b ? a.ref_planes_b + (w0 - REF_SHIFT_WORDS) : a.ref_planes + w0;
#pragma unroll
    for (int w = 0; w <= W; ++w)
        d.win[w] = 32u * w < span ? src[w] : make_uint2(0u, 0u);
}

template <int W>
__device__ __forceinline__ void load_data(const FilterArgs &a, const PairIdx &p, PairData<W> &d)
{
    const uint32_t r = p.r < a.n_reads ? p.r : 0u;
    d.m = a.n_reads ? (uint32_t)ld_once(a, a.read_len + r) : 0u;
#pragma unroll
    for (int j = 0; j < 2 * W; ++j) {
        const uint32_t *row = a.reads + (size_t)j * a.pitch;
        d.words[j] = (a.n_reads && (uint32_t)j < a.rows) ? ld_once(a, row + r) : 0u;
    }
    load_window<W>(a, p.pos, d);
}

// Whether a pair whose loads have arrived can be compared (Sec. 3.3): returns
// PAIR_OK and sets m, or GK_INVALID (read length 0 or above max_read_len, or
// no such read) or GK_UNDEFINED (an unknown base in the read or the window, or
// a window past the reference end).
constexpr uint32_t PAIR_OK = 0xFFu;

template <int W>
__device__ __forceinline__ uint32_t pair_gate(const FilterArgs &a, const PairIdx &p,
                                              const PairData<W> &d, uint32_t &m)
{
    m = p.r < a.n_reads ? d.m : 0u;
    if (m == 0u || m > a.max_read_len)
        return GK_INVALID;
    if ((uint64_t)p.pos + m > a.ref_len || (a.read_has_n && a.read_has_n[p.r]))
        return GK_UNDEFINED;
    if (a.ref_has_unknown && a.ref_unk_lines) {
        // Only windows touching a 512-base line that holds an unknown base
        // read the unknown plane (m <= 512, so at most two lines).
        const uint32_t l0 = p.pos / LINE_BASES, l1 = (p.pos + m - 1u) / LINE_BASES;
        const bool near = ((a.ref_unk_lines[l0 >> 6] >> (l0 & 63u)) |
                           (a.ref_unk_lines[l1 >> 6] >> (l1 & 63u))) & 1ull;
        if (!near)
            return PAIR_OK;
    }
    if (a.ref_has_unknown) {
        const uint32_t s = p.pos & 31u;
        const uint32_t *u = a.ref_unk + (p.pos >> 5);
        uint32_t any = 0, cu = u[0];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint32_t nu = u[w + 1];
            any |= funnel(nu, cu, s) & ones_below((int)m - 32 * w);
            cu = nu;
        }
        if (any)
            return GK_UNDEFINED;
    }
    return PAIR_OK;
}

// Read and window bit-planes of a pair that passed pair_gate: the window
// words are funnel-shifted by pos mod 32 and cleared at or beyond m.
template <int W, int L>
__device__ __forceinline__ void pair_planes(const PairIdx &p, const PairData<W> &d, uint32_t m,
                                            uint32_t (&gh)[W], uint32_t (&gl)[W],
                                            uint32_t (&rh)[W], uint32_t (&rl)[W])
{
    const uint32_t s = p.pos & 31u;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const uint32_t v = ones_below((int)m - 32 * w);
        gh[w] = funnel(d.win[w + 1].x, d.win[w].x, s) & v;
        gl[w] = funnel(d.win[w + 1].y, d.win[w].y, s) & v;
        planes_from_words<L>(d.words[2 * w], d.words[2 * w + 1], rh[w], rl[w]);
    }
}

// Filter one pair whose loads have arrived: returns the result code and sets
// est (GK_EST_NONE unless REJECT / ACCEPT).  With GENERAL false the caller
// guarantees 32(W-1) < m <= 32W and min(e, m-1) <= 31 for every valid pair,
// and only the register-light fast path is compiled.  VAR compiles the
// variant semantics of a.flags (GK_FLAG_*); without it a.flags must be 0, and
// the paper's filter is the only code in the kernel.  KEPT: the read has no
// rows in memory (a.reads is not used), and the general path rebuilds its
// planes from d.words.
template <int W, int L, bool GENERAL = true, bool VAR = false, bool KEPT = false>
__device__ __forceinline__ uint32_t compute_pair(const FilterArgs &a, const PairIdx &p,
                                                 const PairData<W> &d, uint32_t &est)
{
    est = GK_EST_NONE;
    uint32_t m;
    const uint32_t gate = pair_gate<W>(a, p, d, m);
    if (gate != PAIR_OK)
        return gate;
    uint32_t gh[W], gl[W], rh[W], rl[W];
    pair_planes<W, L>(p, d, m, gh, gl, rh, rl);
    const uint32_t kmax = p.e < m - 1u ? p.e : m - 1u;
    const bool exact = !GENERAL || (m > 32u * (W - 1) && kmax <= 31u);
    if (exact) {
        const uint32_t vtop = ones_below((int)m - 32 * (W - 1));
        rh[W - 1] &= vtop;
        rl[W - 1] &= vtop;
    }
    if constexpr (VAR) {                       // variants (uniform per launch)
        if (a.flags & GK_FLAG_HAMMING_FASTPATH) {
            uint32_t hd = 0;
#pragma unroll
            for (int w = 0; w < W; ++w)
                hd += __builtin_popcount(((rh[w] ^ gh[w]) | (rl[w] ^ gl[w])) &
                                         ones_below((int)m - 32 * w));
            if (hd <= p.e) {
                est = hd;
                return GK_ACCEPT;
            }
        }
        if (a.flags & GK_FLAG_NO_REFINE) {
            est = exact ? filter_exact<W, false>(rh, rl, gh, gl, m, kmax)
                        : filter_general<W, L, false, KEPT>(a, p.r, d.words, rh, rl, gh, gl,
                                                                  m, kmax);
            return est <= p.e ? GK_ACCEPT : GK_REJECT;
        }
    }
    est = exact ? filter_exact<W>(rh, rl, gh, gl, m, kmax)
                : filter_general<W, L, true, KEPT>(a, p.r, d.words, rh, rl, gh, gl, m, kmax);
    return est <= p.e ? GK_ACCEPT : GK_REJECT;
}

}  // namespace gkd

// GateKeeper-GPU filter kernel for gfx950 (CDNA4).
//
// One lane per (read, candidate) pair, as the paper assigns one thread per
// filtration (Sec. 3.2).  Unlike the paper's kernel, which keeps 2e+1 masks
// of 2-bit-interleaved words in thread-local stack arrays, this kernel:
//   - holds the read and the window as two bit-planes (high and low code bit)
//     of 32 bases per 32-bit register, so "XOR the codes, OR the two bits"
//     (Sec. 2.1) is (rh ^ gh) | (rl ^ gl) over 32 bases at once;
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
#include "gk_internal.h"

namespace gkd {
namespace {

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

// Three delta swaps on 16 packed 2-bit codes (base j in bits 2j, 2j+1):
// afterwards byte 0 holds the low code bits of bases 0-7, byte 1 their high
// bits, byte 2 the low bits of bases 8-15 and byte 3 their high bits, so two
// byte permutes assemble the 32-base planes.
__device__ __forceinline__ uint32_t unzip3(uint32_t x)
{
    uint32_t t;
    t = (x ^ (x >> 1)) & 0x22222222u; x = x ^ t ^ (t << 1);
    t = (x ^ (x >> 2)) & 0x0C0C0C0Cu; x = x ^ t ^ (t << 2);
    t = (x ^ (x >> 4)) & 0x00F000F0u; x = x ^ t ^ (t << 4);
    return x;
}

// Packed words p0 (bases 0-15) and p1 (bases 16-31) -> bit-planes of 32 bases.
__device__ __forceinline__ void planes_from_packed(uint32_t p0, uint32_t p1, uint32_t &hi,
                                                   uint32_t &lo)
{
    const uint32_t x0 = unzip3(p0), x1 = unzip3(p1);
    lo = __builtin_amdgcn_perm(x1, x0, 0x06040200u);
    hi = __builtin_amdgcn_perm(x1, x0, 0x07050301u);
}

// Read r's plane words 0..W-1 (words at or beyond the read length are 0).
template <int W>
__device__ __forceinline__ void load_read(const FilterArgs &a, uint32_t r, uint32_t m,
                                          uint32_t (&rh)[W], uint32_t (&rl)[W])
{
    const uint32_t *base = a.reads + r;
    const size_t pitch = a.pitch;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const uint32_t p0 = (m > 32u * w) ? base[(2 * w) * pitch] : 0u;
        const uint32_t p1 = (m > 32u * w + 16u) ? base[(2 * w + 1) * pitch] : 0u;
        planes_from_packed(p0, p1, rh[w], rl[w]);
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
// word 0 and those of I_k in words W-2 and W-1.
template <int W>
__device__ __forceinline__ uint32_t filter_exact(uint32_t (&rh)[W], uint32_t (&rl)[W],
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
            Xd[w] = w == 0 ? lead : 0u;
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
        Xi[W - 1] = ~(vtop >> k);
        if (W >= 2)
            Xi[W >= 2 ? W - 2 : 0] = ~funnel(vtop, 0xFFFFFFFFu, k);
        amend_and<W>(M, acc, Xi);
    }

    uint32_t est = 0;
#pragma unroll
    for (int w = 0; w < W; ++w)
        est += __builtin_popcount(acc[w]);
    return est;
}

// General path: any m <= 32W and any k <= m-1 <= 511.  Shifts of 32 bases or
// more move whole words: the read planes are shifted in place by one word each
// time k passes a multiple of 32, and reloaded between the deletion and the
// insertion loop.
template <int W>
__device__ __forceinline__ uint32_t filter_general(const FilterArgs &a, uint32_t r,
                                                uint32_t (&rh)[W], uint32_t (&rl)[W],
                                                const uint32_t (&gh)[W], const uint32_t (&gl)[W],
                                                uint32_t m, uint32_t kmax)
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
            X[w] = ones_below((int)k - 32 * w);
        }
        amend_and<W>(M, acc, X);
    }

    load_read<W>(a, r, m, rh, rl);
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
            X[w] = V[w] & ~ones_below((int)m - (int)k - 32 * w);
        amend_and<W>(M, acc, X);
    }

    uint32_t est = 0;
#pragma unroll
    for (int w = 0; w < W; ++w)
        est += __builtin_popcount(acc[w]);
    return est;
}

template <int W>
__global__ __launch_bounds__(256) void k_filter(FilterArgs a)
{
    const uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    uint32_t res = GK_INVALID;
    if (i < a.n_pairs) {
        uint32_t est = GK_EST_NONE;
        const uint32_t r = a.pair_read[i];
        const uint32_t pos = a.cand_pos[i];
        const uint32_t e = a.e_pair ? (uint32_t)a.e_pair[i] : a.e_uniform;
        const uint32_t m = r < a.n_reads ? (uint32_t)a.read_len[r] : 0u;
        if (m == 0u || m > a.max_read_len) {
            res = GK_INVALID;
        } else if ((uint64_t)pos + m > a.ref_len || (a.read_has_n && a.read_has_n[r])) {
            res = GK_UNDEFINED;
        } else {
            // Window gather: W+1 words per plane from word pos/32, funnel-shifted
            // by pos mod 32.  The reference padding keeps every load in bounds.
            const uint2 *src = a.ref_planes + (pos >> 5);
            const uint32_t s = pos & 31u;
            uint32_t gh[W], gl[W];
            uint2 cur = src[0];
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const uint2 nxt = src[w + 1];
                gh[w] = funnel(nxt.x, cur.x, s);
                gl[w] = funnel(nxt.y, cur.y, s);
                cur = nxt;
            }
            bool unknown = false;
            if (a.ref_has_unknown) {
                const uint32_t *u = a.ref_unk + (pos >> 5);
                uint32_t any = 0, cu = u[0];
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const uint32_t nu = u[w + 1];
                    any |= funnel(nu, cu, s) & ones_below((int)m - 32 * w);
                    cu = nu;
                }
                unknown = any != 0u;
            }
            if (unknown) {
                res = GK_UNDEFINED;
            } else {
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const uint32_t v = ones_below((int)m - 32 * w);
                    gh[w] &= v;
                    gl[w] &= v;
                }
                uint32_t rh[W], rl[W];
                load_read<W>(a, r, m, rh, rl);
                const uint32_t kmax = e < m - 1u ? e : m - 1u;
                if (m > 32u * (W - 1) && kmax <= 31u) {
                    rh[W - 1] &= ones_below((int)m - 32 * (W - 1));
                    rl[W - 1] &= ones_below((int)m - 32 * (W - 1));
                    est = filter_exact<W>(rh, rl, gh, gl, m, kmax);
                } else {
                    est = filter_general<W>(a, r, rh, rl, gh, gl, m, kmax);
                }
                res = est <= e ? GK_ACCEPT : GK_REJECT;
            }
        }
        a.accept[i] = (uint8_t)res;
        a.est[i] = (uint16_t)est;
    }
    if (a.accept_bits) {
        const bool pass = i < a.n_pairs && (res == GK_ACCEPT || res == GK_UNDEFINED);
        const unsigned long long bits = __ballot(pass);
        if ((threadIdx.x & 63u) == 0u && i < a.n_pairs)
            a.accept_bits[i >> 6] = bits;
    }
}

template <int W>
hipError_t launch_w(const FilterArgs &a, hipStream_t s)
{
    const uint64_t blocks = (a.n_pairs + 255u) / 256u;
    hipLaunchKernelGGL(k_filter<W>, dim3((uint32_t)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_filter(const FilterArgs &a, uint32_t words, hipStream_t s)
{
    switch (words) {
    case 1: return launch_w<1>(a, s);
    case 2: return launch_w<2>(a, s);
    case 3: return launch_w<3>(a, s);
    case 4: return launch_w<4>(a, s);
    case 5: return launch_w<5>(a, s);
    case 6: return launch_w<6>(a, s);
    case 7: return launch_w<7>(a, s);
    case 8: return launch_w<8>(a, s);
    case 9: return launch_w<9>(a, s);
    case 10: return launch_w<10>(a, s);
    case 11: return launch_w<11>(a, s);
    case 12: return launch_w<12>(a, s);
    case 13: return launch_w<13>(a, s);
    case 14: return launch_w<14>(a, s);
    case 15: return launch_w<15>(a, s);
    case 16: return launch_w<16>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace gkd

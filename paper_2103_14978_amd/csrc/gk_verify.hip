// Verification of filtered pairs: the exact edit distance (unit-cost global
// alignment of the read and its window, the ground truth of Sec. 4.4) that the
// read mapper's verification step computes for the pairs the filter passes
// (Sec. 3.3, Sec. 3.5), capped at e + 1.
//
// One lane computes one pair with a bit-parallel edit distance restricted to
// the 2e+1 diagonals |i - j| <= e of the dynamic-programming matrix (a path
// leaving them costs more than e).  The band's vertical differences are kept
// in one word of 2e+1 bits (32-bit for e <= 15, 64-bit for e <= 31); per text
// column the band slides down one row and the column step of Myers' bit-vector
// algorithm (in Hyyro's formulation) updates it.  Boundary choices:
//   - rows above row 0 are virtual with D[i][j] = j - i, which keeps
//     D[0][j] = j and satisfies the recurrence whatever they match, so the
//     band slides from the first column on;
//   - the cell above the band takes D[i][j-1] + 1 and the cell entering at
//     the band's bottom takes D[i-1][j] + 1: both bound the true values from
//     above, so every band value is an upper bound, and it is exact along any
//     path of cost <= e;
//   - rows below the read end never influence row m.
// The diagonal cell D[j][j] is tracked through the band's diagonal zero-delta
// bit, and D[m][m] is the result.
#include "gk_pair.h"
#include "gk_verify.h"

namespace gkd {
namespace {

// One column step of the banded edit distance.  bh, bl: the band's read-plane
// bits (bit k = read base j - e + k - 1, 0-based, for text column j); th, tl:
// the text base's code bits as all-zero / all-one masks.
template <typename T>
__device__ __forceinline__ void band_step(T bh, T bl, T th, T tl, T top, T keep, uint32_t e,
                                          T &vp, T &vn, uint32_t &score)
{
    const T eq = ~((bh ^ th) | (bl ^ tl));
    // slide the band down one row; the new bottom row steps +1
    vp = ((vp >> 1) & keep) | top;
    vn = (vn >> 1) & keep;
    const T xv = eq | vn;
    const T xh = (((eq & vp) + vp) ^ vp) | eq;
    score += 1u - (uint32_t)(((xh | vn) >> e) & 1u);   // diagonal step
    T ph = vn | ~(xh | vp);
    T mh = vp & xh;
    ph = (ph << 1) | 1u;                 // the row above the band steps +1
    mh = mh << 1;
    vp = mh | ~(xv | ph);
    vn = ph & xv;
}

// 32 (T = uint32_t) or 64 (T = uint64_t) bits of [a | b | c] from bit s of a.
template <typename T>
__device__ __forceinline__ T bits_from(uint32_t a, uint32_t b, uint32_t c, uint32_t s)
{
    const uint32_t lo = funnel(b, a, s);
    if constexpr (sizeof(T) == 4)
        return lo;
    else
        return ((uint64_t)funnel(c, b, s) << 32) | lo;
}

// Read bases are taken from [32 zero bits | plane words 0..W-1 | zeros]: for
// text column j = 32 blk + c + 1 the band starts at extended bit
// 32 blk + c + 32 - e, which lies in extended word blk (read word blk - 1)
// while c < e and in word blk + 1 (read word blk) from c = e on; the column
// loop is split there so each part reads fixed words.
template <int W, typename T>
__device__ __forceinline__ uint32_t band_distance(const uint32_t (&rh)[W], const uint32_t (&rl)[W],
                                                  const uint32_t (&gh)[W], const uint32_t (&gl)[W],
                                                  uint32_t m, uint32_t e)
{
    const T top = (T)1 << (2 * e);                 // band row 2e: enters each column
    const T keep = top - 1;                        // band rows 0 .. 2e-1 after a slide
    T vn = ((T)2 << e) - 1;                        // column 0: rows -e..0 step -1,
    T vp = (top | keep) & ~vn;                     //           rows 1..e step +1
    uint32_t score = 0;                            // D[j][j]
#pragma unroll
    for (int blk = 0; blk < W; ++blk) {
        const uint32_t h0 = blk >= 1 ? rh[blk - 1] : 0u, l0 = blk >= 1 ? rl[blk - 1] : 0u;
        const uint32_t h1 = rh[blk], l1 = rl[blk];
        const uint32_t h2 = blk + 1 < W ? rh[blk + 1] : 0u, l2 = blk + 1 < W ? rl[blk + 1] : 0u;
        const uint32_t h3 = blk + 2 < W ? rh[blk + 2] : 0u, l3 = blk + 2 < W ? rl[blk + 2] : 0u;
        const int cols = (int)m - 32 * blk < 32 ? (int)m - 32 * blk : 32;
        const int split = (int)e < cols ? (int)e : cols;
        const uint32_t th_w = gh[blk], tl_w = gl[blk];
        for (int c = 0; c < split; ++c) {          // band starts in read word blk - 1
            const uint32_t s = (uint32_t)c + 32u - e;
            band_step<T>(bits_from<T>(h0, h1, h2, s), bits_from<T>(l0, l1, l2, s),
                         (T)(int32_t)__builtin_amdgcn_sbfe(th_w, c, 1),
                         (T)(int32_t)__builtin_amdgcn_sbfe(tl_w, c, 1), top, keep, e, vp, vn,
                         score);
        }
        for (int c = split; c < cols; ++c) {       // band starts in read word blk
            const uint32_t s = (uint32_t)c - e;
            band_step<T>(bits_from<T>(h1, h2, h3, s), bits_from<T>(l1, l2, l3, s),
                         (T)(int32_t)__builtin_amdgcn_sbfe(th_w, c, 1),
                         (T)(int32_t)__builtin_amdgcn_sbfe(tl_w, c, 1), top, keep, e, vp, vn,
                         score);
        }
    }
    return score < e + 1u ? score : e + 1u;
}

template <int W, int L>
__global__ __launch_bounds__(256) void k_verify(FilterArgs a, const uint32_t *list,
                                                const uint32_t *count, uint16_t *dist)
{
    const uint32_t n = *count;
    for (uint32_t t = blockIdx.x * 256u + threadIdx.x; t < n; t += gridDim.x * 256u) {
        const uint32_t i = list[t];
        const PairIdx p = load_idx(a, i);
        PairData<W> d;
        load_data<W>(a, p, d);
        uint32_t m, out = GK_EST_NONE;
        if (p.e <= GK_VERIFY_MAX_E && pair_gate<W>(a, p, d, m) == PAIR_OK) {
            uint32_t gh[W], gl[W], rh[W], rl[W];
            pair_planes<W, L>(p, d, m, gh, gl, rh, rl);
            out = p.e <= 15u ? band_distance<W, uint32_t>(rh, rl, gh, gl, m, p.e)
                             : band_distance<W, uint64_t>(rh, rl, gh, gl, m, p.e);
        }
        dist[i] = (uint16_t)out;
    }
}

__global__ void k_verify_reset(uint32_t *count) { *count = 0u; }

// Lists the pairs to verify (accept[i] == GK_ACCEPT, or every pair when
// accept is NULL) in pair order within each workgroup's contiguous range, with
// one atomic per workgroup: a first pass counts the range's selected pairs, a
// second writes them.  The other pairs get GK_EST_NONE.
__global__ __launch_bounds__(256) void k_verify_select(const uint8_t *accept, uint32_t n,
                                                       uint32_t *list, uint32_t *count,
                                                       uint16_t *dist)
{
    __shared__ uint32_t wave_sum[4];
    __shared__ uint32_t base;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t per = ((n + gridDim.x - 1) / gridDim.x + 255u) & ~255u;
    const uint32_t lo = blockIdx.x * per;
    const uint32_t hi = lo + per < n ? lo + per : n;

    uint32_t c = 0;
    for (uint32_t i = lo + threadIdx.x; i < hi; i += 256u) {
        const bool sel = accept == nullptr || accept[i] == GK_ACCEPT;
        c += sel ? 1u : 0u;
        if (!sel)
            dist[i] = (uint16_t)GK_EST_NONE;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        c += __shfl_xor(c, o, 64);
    if (lane == 0u)
        wave_sum[wave] = c;
    __syncthreads();
    if (threadIdx.x == 0u) {
        const uint32_t total = wave_sum[0] + wave_sum[1] + wave_sum[2] + wave_sum[3];
        base = total ? atomicAdd(count, total) : 0u;
    }
    __syncthreads();
    uint32_t run = base;
    for (uint32_t start = lo; start < hi; start += 256u) {     // uniform per block
        const uint32_t i = start + threadIdx.x;
        const bool sel = i < hi && (accept == nullptr || accept[i] == GK_ACCEPT);
        const unsigned long long mask = __ballot(sel);
        __syncthreads();                 // wave_sum of the previous step is read
        if (lane == 0u)
            wave_sum[wave] = (uint32_t)__popcll(mask);
        __syncthreads();
        uint32_t before = 0;
        for (uint32_t w = 0; w < wave; ++w)
            before += wave_sum[w];
        if (sel)
            list[run + before + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull))] = i;
        run += wave_sum[0] + wave_sum[1] + wave_sum[2] + wave_sum[3];
    }
}

template <int W, int L>
hipError_t verify_wl(const FilterArgs &a, const uint8_t *accept, uint16_t *dist, uint32_t *list,
                     uint32_t *count, int cus, hipStream_t s)
{
    static int per_cu = -1;
    if (per_cu < 0) {
        int v = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_verify<W, L>, 256, 0);
        if (e != hipSuccess)
            return e;
        per_cu = v > 0 ? v : 1;
    }
    const uint64_t CHUNK = 1ull << 30;
    for (uint64_t first = 0; first < a.n_pairs; first += CHUNK) {
        FilterArgs c = a;
        const uint64_t n = a.n_pairs - first < CHUNK ? a.n_pairs - first : CHUNK;
        c.n_pairs = n;
        c.pair_read = a.pair_read ? a.pair_read + first : nullptr;
        c.cand_pos = a.cand_pos + first;
        c.e_pair = a.e_pair ? a.e_pair + first : nullptr;
        c.accept = nullptr;
        c.est = nullptr;
        c.accept_bits = nullptr;
        const uint8_t *acc = accept ? accept + first : nullptr;
        uint16_t *out = dist + first;
        hipLaunchKernelGGL(k_verify_reset, dim3(1), dim3(1), 0, s, count);
        const uint64_t want = (n + 255) / 256;
        const uint32_t sel_blocks = (uint32_t)(want < (uint64_t)cus * 4 ? want : (uint64_t)cus * 4);
        hipLaunchKernelGGL(k_verify_select, dim3(sel_blocks), dim3(256), 0, s, acc, (uint32_t)n,
                           list, count, out);
        const uint64_t vb = want < (uint64_t)cus * per_cu ? want : (uint64_t)cus * per_cu;
        hipLaunchKernelGGL((k_verify<W, L>), dim3((uint32_t)vb), dim3(256), 0, s, c, list, count,
                           out);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

template <int L>
hipError_t verify_l(const FilterArgs &a, const uint8_t *accept, uint16_t *dist, uint32_t *list,
                    uint32_t *count, uint32_t words, int cus, hipStream_t s)
{
    switch (words) {
    case 1: return verify_wl<1, L>(a, accept, dist, list, count, cus, s);
    case 2: return verify_wl<2, L>(a, accept, dist, list, count, cus, s);
    case 3: return verify_wl<3, L>(a, accept, dist, list, count, cus, s);
    case 4: return verify_wl<4, L>(a, accept, dist, list, count, cus, s);
    case 5: return verify_wl<5, L>(a, accept, dist, list, count, cus, s);
    case 6: return verify_wl<6, L>(a, accept, dist, list, count, cus, s);
    case 7: return verify_wl<7, L>(a, accept, dist, list, count, cus, s);
    case 8: return verify_wl<8, L>(a, accept, dist, list, count, cus, s);
    case 9: return verify_wl<9, L>(a, accept, dist, list, count, cus, s);
    case 10: return verify_wl<10, L>(a, accept, dist, list, count, cus, s);
    case 11: return verify_wl<11, L>(a, accept, dist, list, count, cus, s);
    case 12: return verify_wl<12, L>(a, accept, dist, list, count, cus, s);
    case 13: return verify_wl<13, L>(a, accept, dist, list, count, cus, s);
    case 14: return verify_wl<14, L>(a, accept, dist, list, count, cus, s);
    case 15: return verify_wl<15, L>(a, accept, dist, list, count, cus, s);
    case 16: return verify_wl<16, L>(a, accept, dist, list, count, cus, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_verify(const FilterArgs &a, const uint8_t *accept, uint16_t *dist,
                         uint32_t *list, uint32_t *count, uint32_t words, uint32_t layout,
                         int cus, hipStream_t s)
{
    return layout == GK_READS_INTERLEAVED
               ? verify_l<GK_READS_INTERLEAVED>(a, accept, dist, list, count, words, cus, s)
               : verify_l<GK_READS_SPLIT>(a, accept, dist, list, count, words, cus, s);
}

}  // namespace gkd

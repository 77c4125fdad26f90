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

// A 64-bit band word kept as two 32-bit halves, so that chains of logic
// operations on it map onto 3-input logic instructions per half (whole 64-bit
// values get split into halves only after that combining is done).
struct B64 {
    uint32_t lo, hi;
};
__device__ __forceinline__ B64 operator&(B64 a, B64 b) { return {a.lo & b.lo, a.hi & b.hi}; }
__device__ __forceinline__ B64 operator|(B64 a, B64 b) { return {a.lo | b.lo, a.hi | b.hi}; }
__device__ __forceinline__ B64 operator^(B64 a, B64 b) { return {a.lo ^ b.lo, a.hi ^ b.hi}; }
__device__ __forceinline__ B64 operator~(B64 a) { return {~a.lo, ~a.hi}; }
__device__ __forceinline__ B64 operator+(B64 a, B64 b)
{
    const uint64_t s = (((uint64_t)a.hi << 32) | a.lo) + (((uint64_t)b.hi << 32) | b.lo);
    return {(uint32_t)s, (uint32_t)(s >> 32)};
}

template <typename T> __device__ __forceinline__ T from64(uint64_t v);
template <> __device__ __forceinline__ uint32_t from64<uint32_t>(uint64_t v) { return (uint32_t)v; }
template <> __device__ __forceinline__ B64 from64<B64>(uint64_t v)
{
    return {(uint32_t)v, (uint32_t)(v >> 32)};
}

// all-zero / all-one mask of one text code bit
template <typename T> __device__ __forceinline__ T broadcast(uint32_t m);
template <> __device__ __forceinline__ uint32_t broadcast<uint32_t>(uint32_t m) { return m; }
template <> __device__ __forceinline__ B64 broadcast<B64>(uint32_t m) { return {m, m}; }

__device__ __forceinline__ uint32_t shr1(uint32_t x) { return x >> 1; }
__device__ __forceinline__ B64 shr1(B64 x) { return {funnel(x.hi, x.lo, 1), x.hi >> 1}; }

// bit e of x; e <= 31 in both widths (the wide band serves 16 <= e <= 31)
__device__ __forceinline__ uint32_t bit_at(uint32_t x, uint32_t e) { return (x >> e) & 1u; }
__device__ __forceinline__ uint32_t bit_at(B64 x, uint32_t e) { return (x.lo >> e) & 1u; }

// One column step of the banded edit distance.  bh, bl: the band's read-plane
// bits (bit k = read base j - e + k - 1, 0-based, for text column j); th, tl:
// the text base's code bits as all-zero / all-one masks.  vp, vn come in
// already slid down one row into this column's band (bit 2e, the new bottom
// row, steps +1) and leave slid into the next column's: the slide's shift
// right cancels the shift left of the horizontal deltas, so the next column's
// vertical deltas at band row k read the horizontal deltas of row k and the
// XV bit of row k + 1 directly.  Bits above 2e may hold anything in eq, xh, ph
// and mh: carries and shifts only move information upward there, and the
// masks keep them out of vp and vn.
template <typename T>
__device__ __forceinline__ T band_column(T eq, T top, T keep, T &vp, T &vn)
{
    const T xh = (((eq & vp) + vp) ^ vp) | eq;
    const T diag = xh | vn;              // bit e: the diagonal did not step +1
    // Horizontal deltas +1 / -1 of the band rows.  The row above the band
    // (+1) would only enter bit 0 of this column's new vertical deltas, which
    // the slide drops.
    const T ph = vn | ~(xh | vp);
    const T mh = vp & xh;
    const T xv1 = shr1(eq | vn);         // XV of the next column's band rows
    vp = ((mh | ~(xv1 | ph)) & keep) | top;
    vn = ph & xv1 & keep;
    return diag;
}

template <typename T>
__device__ __forceinline__ void band_step(T bh, T bl, T th, T tl, T top, T keep, uint32_t e,
                                          T &vp, T &vn, uint32_t &flat)
{
    const T eq = ~((bh ^ th) | (bl ^ tl));
    flat += bit_at(band_column(eq, top, keep, vp, vn), e);
}

// 32 (T = uint32_t) or 64 (T = B64) bits of [a | b | c] from bit s of a.
template <typename T>
__device__ __forceinline__ T bits_from(uint32_t a, uint32_t b, uint32_t c, uint32_t s)
{
    const uint32_t lo = funnel(b, a, s);
    if constexpr (sizeof(T) == 4)
        return lo;
    else
        return B64{lo, funnel(c, b, s)};
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
    const uint64_t top64 = 1ull << (2 * e);        // band row 2e: enters each column
    const uint64_t keep64 = top64 - 1;             // band rows 0 .. 2e-1 after a slide
    const uint64_t vn0 = (2ull << e) - 1;          // column 0: rows -e..0 step -1,
    const uint64_t vp0 = (top64 | keep64) & ~vn0;  //           rows 1..e step +1
    const T top = from64<T>(top64), keep = from64<T>(keep64);
    T vp = from64<T>(((vp0 >> 1) & keep64) | top64);   // slid into column 1's band
    T vn = from64<T>((vn0 >> 1) & keep64);
    uint32_t flat = 0;                             // columns j where D[j][j] = D[j-1][j-1]
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
                         broadcast<T>(__builtin_amdgcn_sbfe(th_w, c, 1)),
                         broadcast<T>(__builtin_amdgcn_sbfe(tl_w, c, 1)), top, keep, e, vp, vn,
                         flat);
        }
        for (int c = split; c < cols; ++c) {       // band starts in read word blk
            const uint32_t s = (uint32_t)c - e;
            band_step<T>(bits_from<T>(h1, h2, h3, s), bits_from<T>(l1, l2, l3, s),
                         broadcast<T>(__builtin_amdgcn_sbfe(th_w, c, 1)),
                         broadcast<T>(__builtin_amdgcn_sbfe(tl_w, c, 1)), top, keep, e, vp, vn,
                         flat);
        }
    }
    const uint32_t score = m - flat;               // D[m][m]: each diagonal step is 0 or +1
    return score < e + 1u ? score : e + 1u;
}

// Two pairs with the same length m and the same e <= 7 in one 32-bit word:
// pair 0's band in bits 0..15, pair 1's in bits 16..31.  A band of 2e+1 <= 15
// rows keeps (eq & vp) + vp below 2^(2e+2) <= 2^16, so no carry crosses into
// the other pair's half; the shift right moves bit 16 into half 0's bit 15,
// above its band, where the masks clear it.  Both pairs share every logic
// instruction; only the gathers of their read bits and text bits are
// separate (byte permutes put the two halves together).  Returns
// dist0 | dist1 << 16.
__device__ __forceinline__ uint32_t halves(uint32_t hi_src, uint32_t lo_src)
{
    return __builtin_amdgcn_perm(hi_src, lo_src, 0x05040100u);   // {lo_src[15:0], hi_src[15:0]}
}

// One column of both pairs: h0, l0 / h1, l1 are 32 read-plane bits from each
// pair's band start; the text bits are bit c of each pair's window words.
__device__ __forceinline__ void band_step2(uint32_t h0, uint32_t l0, uint32_t h1, uint32_t l1,
                                           uint32_t t0h, uint32_t t0l, uint32_t t1h,
                                           uint32_t t1l, int c, uint32_t top, uint32_t keep,
                                           uint32_t e, uint32_t &vp, uint32_t &vn,
                                           uint32_t &flat)
{
    const uint32_t bh = halves(h1, h0), bl = halves(l1, l0);
    const uint32_t th = halves((uint32_t)__builtin_amdgcn_sbfe(t1h, c, 1),
                               (uint32_t)__builtin_amdgcn_sbfe(t0h, c, 1));
    const uint32_t tl = halves((uint32_t)__builtin_amdgcn_sbfe(t1l, c, 1),
                               (uint32_t)__builtin_amdgcn_sbfe(t0l, c, 1));
    const uint32_t eq = ~((bh ^ th) | (bl ^ tl));
    flat += (band_column<uint32_t>(eq, top, keep, vp, vn) >> e) & 0x00010001u;
}

template <int W>
__device__ __forceinline__ uint32_t band_distance2(
    const uint32_t (&rh0)[W], const uint32_t (&rl0)[W], const uint32_t (&gh0)[W],
    const uint32_t (&gl0)[W], const uint32_t (&rh1)[W], const uint32_t (&rl1)[W],
    const uint32_t (&gh1)[W], const uint32_t (&gl1)[W], uint32_t m, uint32_t e)
{
    const uint32_t top1 = 1u << (2 * e), keep1 = top1 - 1u;
    const uint32_t vn0 = (2u << e) - 1u, vp0 = (top1 | keep1) & ~vn0;
    const uint32_t vps = ((vp0 >> 1) & keep1) | top1, vns = (vn0 >> 1) & keep1;
    const uint32_t top = top1 | (top1 << 16), keep = keep1 | (keep1 << 16);
    uint32_t vp = vps | (vps << 16), vn = vns | (vns << 16);
    uint32_t flat = 0;                   // two 16-bit counters
#pragma unroll
    for (int blk = 0; blk < W; ++blk) {
        const uint32_t a0 = blk >= 1 ? rh0[blk - 1] : 0u, b0 = blk >= 1 ? rl0[blk - 1] : 0u;
        const uint32_t c0 = blk >= 1 ? rh1[blk - 1] : 0u, d0 = blk >= 1 ? rl1[blk - 1] : 0u;
        const uint32_t a1 = rh0[blk], b1 = rl0[blk], c1 = rh1[blk], d1 = rl1[blk];
        const uint32_t a2 = blk + 1 < W ? rh0[blk + 1] : 0u, b2 = blk + 1 < W ? rl0[blk + 1] : 0u;
        const uint32_t c2 = blk + 1 < W ? rh1[blk + 1] : 0u, d2 = blk + 1 < W ? rl1[blk + 1] : 0u;
        const int cols = (int)m - 32 * blk < 32 ? (int)m - 32 * blk : 32;
        const int split = (int)e < cols ? (int)e : cols;
        const uint32_t t0h = gh0[blk], t0l = gl0[blk], t1h = gh1[blk], t1l = gl1[blk];
        for (int c = 0; c < split; ++c)          // band starts in read word blk - 1
            band_step2(funnel(a1, a0, (uint32_t)c + 32u - e), funnel(b1, b0, (uint32_t)c + 32u - e),
                       funnel(c1, c0, (uint32_t)c + 32u - e), funnel(d1, d0, (uint32_t)c + 32u - e),
                       t0h, t0l, t1h, t1l, c, top, keep, e, vp, vn, flat);
        for (int c = split; c < cols; ++c)       // band starts in read word blk
            band_step2(funnel(a2, a1, (uint32_t)c - e), funnel(b2, b1, (uint32_t)c - e),
                       funnel(c2, c1, (uint32_t)c - e), funnel(d2, d1, (uint32_t)c - e),
                       t0h, t0l, t1h, t1l, c, top, keep, e, vp, vn, flat);
    }
    const uint32_t s0 = m - (flat & 0xFFFFu), s1 = m - (flat >> 16);
    return (s0 < e + 1u ? s0 : e + 1u) | ((s1 < e + 1u ? s1 : e + 1u) << 16);
}

// Distance of one pair that passed the gate.  When every active lane has the
// same threshold and length (always so for one read length and a uniform e),
// the band's shifts and trip counts come from scalar registers.
template <int W, int L>
__device__ __forceinline__ uint32_t verify_pair(const PairIdx &p, const PairData<W> &d,
                                                uint32_t m)
{
    uint32_t gh[W], gl[W], rh[W], rl[W];
    pair_planes<W, L>(p, d, m, gh, gl, rh, rl);
    const uint32_t e0 = __builtin_amdgcn_readfirstlane(p.e);
    const uint32_t m0 = __builtin_amdgcn_readfirstlane(m);
    if (__ballot(p.e != e0 || m != m0) == 0ull)
        return e0 <= 15u ? band_distance<W, uint32_t>(rh, rl, gh, gl, m0, e0)
                         : band_distance<W, B64>(rh, rl, gh, gl, m0, e0);
    return p.e <= 15u ? band_distance<W, uint32_t>(rh, rl, gh, gl, m, p.e)
                      : band_distance<W, B64>(rh, rl, gh, gl, m, p.e);
}

// A pair's loads as load_data does them, but with the read's words taken
// from a row-major copy of the reads (read r's rows at rm[r * rm_stride ..],
// rm_stride a multiple of 4 words, zero past the rows): one read is one run
// of 16-byte loads from one or two lines, instead of a line per row of the
// transposed layout (whose rows only share lines between neighbouring reads).
template <int W>
__device__ __forceinline__ void load_data_rm(const FilterArgs &a, const PairIdx &p,
                                             PairData<W> &d, const uint32_t *rm,
                                             uint32_t rm_stride)
{
    const uint32_t r = p.r < a.n_reads ? p.r : 0u;
    const uint32_t pos = p.pos < a.ref_len ? p.pos : 0u;
    d.m = a.n_reads ? (uint32_t)a.read_len[r] : 0u;
    const uint4 *q = reinterpret_cast<const uint4 *>(rm + (size_t)r * rm_stride);
#pragma unroll
    for (int j = 0; j < 2 * W; j += 4) {
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (a.n_reads && (uint32_t)j < a.rows)
            v = q[j / 4];
        const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (j + k < 2 * W)
                d.words[j + k] = w4[k];
    }
    // the window, as load_data takes it
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

// Transposed read rows (word j of read r at reads[j * pitch + r]) to the
// row-major copy load_data_rm takes: a workgroup stages 256 reads' rows in
// LDS (each row read with consecutive lanes on consecutive words) and each
// lane writes its read's rm_stride words as 16-byte stores (consecutive lanes,
// consecutive reads).
__global__ __launch_bounds__(256) void k_reads_rowmajor(const uint32_t *reads, uint32_t pitch,
                                                        uint32_t rows, uint32_t n_reads,
                                                        uint32_t rm_stride, uint32_t *rm)
{
    extern __shared__ uint32_t rm_lds[];
    const uint32_t t = threadIdx.x;
    const uint32_t r0 = blockIdx.x * 256u;
    const uint32_t r = r0 + t;
    const uint32_t ld = rm_stride + 1u;      // odd pitch: a row's words hit distinct banks
    for (uint32_t j = 0; j < rows; ++j)
        rm_lds[t * ld + j] = r < n_reads ? reads[(size_t)j * pitch + r] : 0u;
    for (uint32_t j = rows; j < rm_stride; ++j)
        rm_lds[t * ld + j] = 0u;
    __syncthreads();
    if (r < n_reads) {
        uint4 *out = reinterpret_cast<uint4 *>(rm + (size_t)r * rm_stride);
        for (uint32_t j = 0; j < rm_stride; j += 4)
            out[j / 4] = make_uint4(rm_lds[t * ld + j], rm_lds[t * ld + j + 1],
                                    rm_lds[t * ld + j + 2], rm_lds[t * ld + j + 3]);
    }
}

// Persistent over the list, one pair per lane; RM: the reads come from the
// row-major copy rm (load_data_rm).
template <int W, int L, bool RM = false>
__global__ __launch_bounds__(256) void k_verify(FilterArgs a, const uint32_t *list,
                                                const uint32_t *count, uint16_t *dist,
                                                const uint32_t *rm = nullptr,
                                                uint32_t rm_stride = 0)
{
    const uint32_t n = *count;
    const uint32_t stride = gridDim.x * 256u;
    for (uint32_t t = blockIdx.x * 256u + threadIdx.x; t < n; t += stride) {
        const uint32_t i = list[t];
        const PairIdx p = load_idx(a, i);
        PairData<W> d;
        if constexpr (RM)
            load_data_rm<W>(a, p, d, rm, rm_stride);
        else
            load_data<W>(a, p, d);
        uint32_t m, out = GK_EST_NONE;
        if (p.e <= GK_VERIFY_MAX_E && pair_gate<W>(a, p, d, m) == PAIR_OK)
            out = verify_pair<W, L>(p, d, m);
        dist[i] = (uint16_t)out;
    }
}

// Persistent over the list, two entries per lane per step (t and t + 64),
// for batches with one e <= 7 and reads of up to 8 words.  When every pair of
// the wave that passes the gate has the length and e of the wave's first such
// pair, each lane's two pairs share a 32-bit band word (band_distance2); pairs
// that fail the gate get GK_EST_NONE.  Otherwise the wave appends its pairs to
// `deferred` (one atomic per wave) for k_verify to do one per lane.  Keeping
// that fallback out of this kernel keeps its registers low (two pairs' planes
// already fill most of them).
template <int W, int L>
__global__ __launch_bounds__(256) void k_verify_paired(FilterArgs a, const uint32_t *list,
                                                       const uint32_t *count, uint16_t *dist,
                                                       uint32_t *deferred,
                                                       uint32_t *deferred_count)
{
    const uint32_t n = *count;
    const uint32_t lane = threadIdx.x & 63u;
    // A wave takes blocks of 128 consecutive list entries, a lane entries
    // lane and lane + 64 of the block: the list orders each listing group by
    // read length, so the two halves of a block mostly share one.
    const uint32_t first = (blockIdx.x * 4u + (threadIdx.x >> 6)) * 128u + lane;
    const uint32_t step = gridDim.x * 4u * 128u;
    for (uint32_t t = first; t < n; t += step) {
        const bool has1 = t + 64u < n;
        const uint32_t i0 = list[t];
        const uint32_t i1 = has1 ? list[t + 64u] : i0;
        const PairIdx p0 = load_idx(a, i0);
        const PairIdx p1 = load_idx(a, i1);
        PairData<W> d0, d1;
        load_data<W>(a, p0, d0);
        load_data<W>(a, p1, d1);
        uint32_t m0 = 0, m1 = 0;
        const bool ok0 = p0.e <= GK_VERIFY_MAX_E && pair_gate<W>(a, p0, d0, m0) == PAIR_OK;
        const bool ok1 = p1.e <= GK_VERIFY_MAX_E && pair_gate<W>(a, p1, d1, m1) == PAIR_OK;
        // the wave's length and e: those of its first pair that passed the gate
        const unsigned long long v0 = __ballot(ok0), v1 = __ballot(ok1);
        uint32_t ew = 0, mw = 0;
        if (v0) {
            const int src = __builtin_ctzll(v0);
            ew = (uint32_t)__builtin_amdgcn_readlane((int)p0.e, src);
            mw = (uint32_t)__builtin_amdgcn_readlane((int)m0, src);
        } else if (v1) {
            const int src = __builtin_ctzll(v1);
            ew = (uint32_t)__builtin_amdgcn_readlane((int)p1.e, src);
            mw = (uint32_t)__builtin_amdgcn_readlane((int)m1, src);
        }
        const bool fits = (!ok0 || (p0.e == ew && m0 == mw)) && (!ok1 || (p1.e == ew && m1 == mw));
        if ((v0 | v1) == 0ull) {
            dist[i0] = (uint16_t)GK_EST_NONE;
            if (has1)
                dist[i1] = (uint16_t)GK_EST_NONE;
        } else if (ew <= 7u && __ballot(!fits) == 0ull) {
            uint32_t gh0[W], gl0[W], rh0[W], rl0[W], gh1[W], gl1[W], rh1[W], rl1[W];
            pair_planes<W, L>(p0, d0, mw, gh0, gl0, rh0, rl0);
            pair_planes<W, L>(p1, d1, mw, gh1, gl1, rh1, rl1);
            const uint32_t two = band_distance2<W>(rh0, rl0, gh0, gl0, rh1, rl1, gh1, gl1, mw, ew);
            dist[i0] = (uint16_t)(ok0 ? (two & 0xFFFFu) : GK_EST_NONE);
            if (has1)
                dist[i1] = (uint16_t)(ok1 ? (two >> 16) : GK_EST_NONE);
        } else {
            const unsigned long long act = __ballot(true), two = __ballot(has1);
            const uint32_t n_act = (uint32_t)__popcll(act), n_two = (uint32_t)__popcll(two);
            uint32_t base = 0;
            if (lane == (uint32_t)__builtin_ctzll(act))
                base = atomicAdd(deferred_count, n_act + n_two);
            base = (uint32_t)__builtin_amdgcn_readlane((int)base, __builtin_ctzll(act));
            const unsigned long long below = (1ull << lane) - 1ull;
            deferred[base + (uint32_t)__popcll(act & below)] = i0;
            if (has1)
                deferred[base + n_act + (uint32_t)__popcll(two & below)] = i1;
        }
    }
}

// Listing the pairs to verify (accept[i] == GK_ACCEPT, or every pair when
// accept is NULL) without a contended counter: a workgroup covers 4096
// consecutive pairs, 16 per lane (one 16-byte load of accept when VEC);
// k_select_count stores each workgroup's count, k_select_scan turns the
// counts into offsets (and the total into *count), k_select_write puts each
// workgroup's pairs at its offset through LDS: in pair order when they all
// have one sort key, else ordered by key (read length; with a per-pair e,
// also whether e > 15), so that the waves of the verify kernels see one
// length and one band width (their fast paths need it).  VEC needs accept
// and dist aligned to 16 bytes; the host checks.
constexpr uint32_t SEL_PER_LANE = 16u, SEL_PER_GROUP = 256u * SEL_PER_LANE;

// Bit j of the result: pair i0 + j is listed.  With fill, the 16 dist entries
// are set to GK_EST_NONE first (k_verify overwrites the listed ones later).
template <bool VEC>
__device__ __forceinline__ uint32_t select_bits(const uint8_t *accept, uint32_t n, uint32_t i0,
                                                uint16_t *dist, bool fill)
{
    const uint32_t valid = i0 < n ? (n - i0 < SEL_PER_LANE ? n - i0 : SEL_PER_LANE) : 0u;
    uint32_t sel = 0;
    if (accept == nullptr) {
        sel = valid == SEL_PER_LANE ? 0xFFFFu : ((1u << valid) - 1u);
    } else if (VEC && valid == SEL_PER_LANE) {
        const uint4 v = *reinterpret_cast<const uint4 *>(accept + i0);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                sel |= (((w[q] >> (8 * b)) & 0xFFu) == GK_ACCEPT ? 1u : 0u) << (4 * q + b);
        if (fill) {
            const uint4 none = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
            reinterpret_cast<uint4 *>(dist + i0)[0] = none;
            reinterpret_cast<uint4 *>(dist + i0)[1] = none;
        }
    } else {
        for (uint32_t j = 0; j < valid; ++j) {
            sel |= (accept[i0 + j] == GK_ACCEPT ? 1u : 0u) << j;
            if (fill)
                dist[i0 + j] = (uint16_t)GK_EST_NONE;
        }
    }
    return sel;
}

template <bool VEC>
__global__ __launch_bounds__(256) void k_select_count(const uint8_t *accept, uint32_t n,
                                                      uint32_t *group_count, uint16_t *dist)
{
    __shared__ uint32_t wave_sum[4];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t i0 = blockIdx.x * SEL_PER_GROUP + threadIdx.x * SEL_PER_LANE;
    uint32_t c = (uint32_t)__popc(select_bits<VEC>(accept, n, i0, dist, true));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        c += __shfl_xor(c, o, 64);
    if (lane == 0u)
        wave_sum[wave] = c;
    __syncthreads();
    if (threadIdx.x == 0u)
        group_count[blockIdx.x] = wave_sum[0] + wave_sum[1] + wave_sum[2] + wave_sum[3];
}

// One workgroup of 1024 lanes: exclusive prefix sums of groups (<= 2^18)
// counts in place, the total into count[0] and 0 into count[1].
__global__ __launch_bounds__(1024) void k_select_scan(uint32_t *group_count, uint32_t groups,
                                                      uint32_t *count)
{
    __shared__ uint32_t wave_sum[16];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t per = (groups + 1023u) / 1024u;
    const uint32_t lo = threadIdx.x * per;
    const uint32_t hi = lo + per < groups ? lo + per : groups;
    uint32_t sum = 0;
    for (uint32_t i = lo; i < hi; ++i)
        sum += group_count[i];
    uint32_t incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(incl, o, 64);
        if (lane >= (uint32_t)o)
            incl += t;
    }
    if (lane == 63u)
        wave_sum[wave] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t w = 0; w < wave; ++w)
        before += wave_sum[w];
    uint32_t run = before + incl - sum;
    for (uint32_t i = lo; i < hi; ++i) {
        const uint32_t v = group_count[i];
        group_count[i] = run;
        run += v;
    }
    if (threadIdx.x == 1023u) {
        count[0] = before + incl;
        count[1] = 0u;               // k_verify_paired's deferred pairs
    }
}

// Sort keys of the 16 pairs i0 .. i0 + 15 a lane lists (bit j of sel): the
// read length when a pair can be compared at it (1..max_read_len), else 0 (it
// fails the gate); with a per-pair e, twice that plus whether e > 15.  With no pair-to-read map the 16 lengths are consecutive
// and come in two 16-byte loads when aligned.
__device__ __forceinline__ void length_keys(const FilterArgs &a, uint32_t i0, uint32_t sel,
                                            uint32_t (&key)[SEL_PER_LANE])
{
    if (a.pair_read == nullptr && i0 + SEL_PER_LANE <= a.n_reads &&
        ((uintptr_t)(a.read_len + i0) & 15u) == 0u) {
        const uint4 v0 = *reinterpret_cast<const uint4 *>(a.read_len + i0);
        const uint4 v1 = *reinterpret_cast<const uint4 *>(a.read_len + i0 + 8);
        const uint32_t w[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
        for (uint32_t j = 0; j < SEL_PER_LANE; ++j)
            key[j] = (w[j >> 1] >> (16u * (j & 1u))) & 0xFFFFu;
    } else if (a.pair_read != nullptr && sel != 0u && i0 + SEL_PER_LANE <= a.n_pairs &&
               ((uintptr_t)(a.pair_read + i0) & 15u) == 0u) {
        // the 16 read indices in four 16-byte loads (one 64-byte span), the
        // lengths of the listed pairs only
        uint32_t r[SEL_PER_LANE];
#pragma unroll
        for (uint32_t q = 0; q < 4u; ++q) {
            const uint4 v = *reinterpret_cast<const uint4 *>(a.pair_read + i0 + 4u * q);
            r[4u * q] = v.x;
            r[4u * q + 1u] = v.y;
            r[4u * q + 2u] = v.z;
            r[4u * q + 3u] = v.w;
        }
#pragma unroll
        for (uint32_t j = 0; j < SEL_PER_LANE; ++j)
            key[j] = (sel & (1u << j)) && r[j] < a.n_reads ? (uint32_t)a.read_len[r[j]] : 0u;
    } else {
#pragma unroll
        for (uint32_t j = 0; j < SEL_PER_LANE; ++j) {
            key[j] = 0u;
            if (sel & (1u << j)) {
                const uint32_t r = a.pair_read ? a.pair_read[i0 + j] : i0 + j;
                key[j] = r < a.n_reads ? (uint32_t)a.read_len[r] : 0u;
            }
        }
    }
#pragma unroll
    for (uint32_t j = 0; j < SEL_PER_LANE; ++j)
        key[j] = key[j] <= a.max_read_len ? key[j] : 0u;
    // With a per-pair e, pairs on the 32-bit band (e <= 15) and on the 64-bit
    // one are kept apart too, so that a wave runs one band width.
    if (a.e_pair) {
#pragma unroll
        for (uint32_t j = 0; j < SEL_PER_LANE; ++j)
            key[j] = 2u * key[j] + ((sel & (1u << j)) && a.e_pair[i0 + j] > 15u ? 1u : 0u);
    }
}

template <bool VEC>
__global__ __launch_bounds__(256) void k_select_write(FilterArgs a, const uint8_t *accept,
                                                      uint32_t n, const uint32_t *group_offset,
                                                      uint32_t *list)
{
    // stage[t]: sort key << 12 | the pair's offset in the group (< 4096)
    __shared__ uint32_t stage[SEL_PER_GROUP];
    __shared__ uint32_t hist[2u * GK_MAX_READ_LEN + 2u];
    __shared__ uint32_t wave_sum[4], wave_min[4], wave_max[4];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t i0 = blockIdx.x * SEL_PER_GROUP + threadIdx.x * SEL_PER_LANE;
    const uint32_t sel = select_bits<VEC>(accept, n, i0, nullptr, false);
    uint32_t k16[SEL_PER_LANE];
    length_keys(a, i0, sel, k16);
    const uint32_t c = (uint32_t)__popc(sel);
    uint32_t incl = c, lo = 0xFFFFFFFFu, hi = 0u;
#pragma unroll
    for (uint32_t j = 0; j < SEL_PER_LANE; ++j)
        if (sel & (1u << j)) {
            lo = k16[j] < lo ? k16[j] : lo;
            hi = k16[j] > hi ? k16[j] : hi;
        }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(incl, o, 64);
        if (lane >= (uint32_t)o)
            incl += t;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t ol = __shfl_xor(lo, o, 64), oh = __shfl_xor(hi, o, 64);
        lo = ol < lo ? ol : lo;
        hi = oh > hi ? oh : hi;
    }
    if (lane == 63u)
        wave_sum[wave] = incl;
    if (lane == 0u) {
        wave_min[wave] = lo;
        wave_max[wave] = hi;
    }
    __syncthreads();
    const uint32_t total = wave_sum[0] + wave_sum[1] + wave_sum[2] + wave_sum[3];
    uint32_t at = incl - c;
    for (uint32_t w = 0; w < wave; ++w)
        at += wave_sum[w];
    const uint32_t g0 = blockIdx.x * SEL_PER_GROUP;
#pragma unroll
    for (uint32_t j = 0; j < SEL_PER_LANE; ++j)
        if (sel & (1u << j))
            stage[at++] = (k16[j] << 12) | (i0 + j - g0);
    uint32_t kmin = wave_min[0], kmax = wave_max[0];
    for (uint32_t w = 1; w < 4u; ++w) {
        kmin = wave_min[w] < kmin ? wave_min[w] : kmin;
        kmax = wave_max[w] > kmax ? wave_max[w] : kmax;
    }
    const uint32_t nb = kmin < kmax ? kmax - kmin + 1u : 0u;
    for (uint32_t b = threadIdx.x; b < nb; b += 256u)
        hist[b] = 0u;
    __syncthreads();
    const uint32_t base = group_offset[blockIdx.x];
    if (nb == 0u) {                      // one key (or nothing listed): pair order
        for (uint32_t t = threadIdx.x; t < total; t += 256u)
            list[base + t] = g0 + (stage[t] & 4095u);
        return;
    }
    // Counting sort by key over [kmin, kmax] (the order within a key does not
    // matter: every result is written at its own pair index).
    for (uint32_t t = threadIdx.x; t < total; t += 256u)
        atomicAdd(&hist[(stage[t] >> 12) - kmin], 1u);
    __syncthreads();
    if (wave == 0u) {                    // exclusive prefix sums of the buckets
        const uint32_t per = (nb + 63u) / 64u;
        const uint32_t b0 = lane * per < nb ? lane * per : nb;
        const uint32_t b1 = b0 + per < nb ? b0 + per : nb;
        uint32_t sum = 0;
        for (uint32_t b = b0; b < b1; ++b)
            sum += hist[b];
        uint32_t run = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(run, o, 64);
            if (lane >= (uint32_t)o)
                run += t;
        }
        run -= sum;
        for (uint32_t b = b0; b < b1; ++b) {
            const uint32_t v = hist[b];
            hist[b] = run;
            run += v;
        }
    }
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < total; t += 256u) {
        const uint32_t v = stage[t];
        list[base + atomicAdd(&hist[(v >> 12) - kmin], 1u)] = g0 + (v & 4095u);
    }
}

// ---- listing by (read length in words, e) over the whole batch ----------
//
// With a threshold per pair, a wave of the one-pair-per-lane kernel takes its
// scalar path (one band width, one shift schedule, scalar trip counts) only
// if its pairs share e and the read length.  After the filter a 4096-pair
// group lists a few hundred pairs over as many (length, e) combinations, so
// sorting within groups leaves nearly every wave mixed.  These kernels sort
// the listed pairs of the whole batch by key = (ceil(m / 32) - 1) * 32 +
// min(e, 31) (512 keys; within a key the lengths differ in the last word
// only): each group counts its pairs per key in LDS and adds the counts to
// one of BIN_COPIES copies of the key counts (by group number, so that no
// count is added to by more than 1 / BIN_COPIES of the groups); a scan turns
// the counts into starts, key-major and copy-minor; each group then reserves
// its run in its copy of each key with one atomic and writes its pairs there
// (the order within a key does not matter: every result is written at its
// own pair index).
constexpr uint32_t NKEYS = 512u;
constexpr uint32_t BIN_COPIES = 32u;
constexpr uint32_t BIN_CELLS = NKEYS * BIN_COPIES;   // counts, then cursors, then starts

__device__ __forceinline__ void bin_keys(const FilterArgs &a, uint32_t i0, uint32_t sel,
                                         uint32_t (&key)[SEL_PER_LANE])
{
    FilterArgs la = a;
    la.e_pair = nullptr;                 // plain read lengths
    uint32_t len[SEL_PER_LANE];
    length_keys(la, i0, sel, len);
#pragma unroll
    for (uint32_t j = 0; j < SEL_PER_LANE; ++j) {
        const uint32_t e = (sel & (1u << j)) ? (uint32_t)a.e_pair[i0 + j] : 0u;
        key[j] = len[j] ? ((len[j] + 31u) / 32u - 1u) * 32u + (e < 31u ? e : 31u) : 0u;
    }
}

// counts and cursors to zero
__global__ __launch_bounds__(256) void k_bin_zero(uint32_t *bins)
{
    for (uint32_t b = blockIdx.x * 256u + threadIdx.x; b < 2u * BIN_CELLS; b += gridDim.x * 256u)
        bins[b] = 0u;
}

template <bool VEC>
__global__ __launch_bounds__(256) void k_bin_count(FilterArgs a, const uint8_t *accept,
                                                   uint32_t n, uint32_t *bins, uint16_t *dist)
{
    __shared__ uint32_t h[NKEYS];
    for (uint32_t b = threadIdx.x; b < NKEYS; b += 256u)
        h[b] = 0u;
    __syncthreads();
    const uint32_t i0 = blockIdx.x * SEL_PER_GROUP + threadIdx.x * SEL_PER_LANE;
    const uint32_t sel = select_bits<VEC>(accept, n, i0, dist, true);
    uint32_t key[SEL_PER_LANE];
    bin_keys(a, i0, sel, key);
#pragma unroll
    for (uint32_t j = 0; j < SEL_PER_LANE; ++j)
        if (sel & (1u << j))
            atomicAdd(&h[key[j]], 1u);
    __syncthreads();
    uint32_t *copy = bins + (blockIdx.x % BIN_COPIES) * NKEYS;
    for (uint32_t b = threadIdx.x; b < NKEYS; b += 256u)
        if (h[b])
            atomicAdd(&copy[b], h[b]);
}

// Starts of every (key, copy) cell, key-major: bins[2 BIN_CELLS + c * NKEYS +
// b] for copy c of key b; count[0] = the total, count[1] = 0.
__global__ __launch_bounds__(1024) void k_bin_scan(uint32_t *bins, uint32_t *count)
{
    __shared__ uint32_t wave_sum[16];
    constexpr uint32_t PER = BIN_CELLS / 1024u;       // cells per thread, key-major
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    uint32_t local[PER], sum = 0;
#pragma unroll
    for (uint32_t q = 0; q < PER; ++q) {
        const uint32_t cell = threadIdx.x * PER + q;  // = key * BIN_COPIES + copy
        local[q] = bins[(cell % BIN_COPIES) * NKEYS + cell / BIN_COPIES];
        sum += local[q];
    }
    uint32_t incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(incl, o, 64);
        if (lane >= (uint32_t)o)
            incl += t;
    }
    if (lane == 63u)
        wave_sum[wave] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t w = 0; w < wave; ++w)
        before += wave_sum[w];
    uint32_t run = before + incl - sum;
#pragma unroll
    for (uint32_t q = 0; q < PER; ++q) {
        const uint32_t cell = threadIdx.x * PER + q;
        bins[2u * BIN_CELLS + (cell % BIN_COPIES) * NKEYS + cell / BIN_COPIES] = run;
        run += local[q];
    }
    if (threadIdx.x == 1023u) {
        count[0] = before + incl;
        count[1] = 0u;
    }
}

template <bool VEC>
__global__ __launch_bounds__(256) void k_bin_write(FilterArgs a, const uint8_t *accept,
                                                   uint32_t n, uint32_t *bins, uint32_t *list)
{
    __shared__ uint32_t h[NKEYS];
    for (uint32_t b = threadIdx.x; b < NKEYS; b += 256u)
        h[b] = 0u;
    __syncthreads();
    const uint32_t i0 = blockIdx.x * SEL_PER_GROUP + threadIdx.x * SEL_PER_LANE;
    const uint32_t sel = select_bits<VEC>(accept, n, i0, nullptr, false);
    uint32_t key[SEL_PER_LANE], rank[SEL_PER_LANE];
    bin_keys(a, i0, sel, key);
#pragma unroll
    for (uint32_t j = 0; j < SEL_PER_LANE; ++j)
        rank[j] = (sel & (1u << j)) ? atomicAdd(&h[key[j]], 1u) : 0u;
    __syncthreads();
    // this group's run in its copy of each key: the cell's start plus a
    // reservation on the cell's cursor
    const uint32_t c = (blockIdx.x % BIN_COPIES) * NKEYS;
    for (uint32_t b = threadIdx.x; b < NKEYS; b += 256u)
        if (h[b])
            h[b] = bins[2u * BIN_CELLS + c + b] + atomicAdd(&bins[BIN_CELLS + c + b], h[b]);
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < SEL_PER_LANE; ++j)
        if (sel & (1u << j))
            list[h[key[j]] + rank[j]] = i0 + j;
}

// Resident 256-lane workgroups per CU of k_verify (PAIRED false) or
// k_verify_paired (true).
template <int W, int L, bool PAIRED, bool RM = false>
hipError_t verify_blocks_per_cu(int &out)
{
    static int per_cu = -1;
    if (per_cu < 0) {
        int v = 0;
        hipError_t e = PAIRED ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                    &v, k_verify_paired<W, L>, 256, 0)
                              : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                    &v, k_verify<W, L, RM>, 256, 0);
        if (e != hipSuccess)
            return e;
        per_cu = v > 0 ? v : 1;
    }
    out = per_cu;
    return hipSuccess;
}

template <int W, int L>
hipError_t verify_wl(const FilterArgs &a, const uint8_t *accept, uint16_t *dist, uint32_t *list,
                     uint32_t *groups_buf, uint32_t *deferred, uint32_t *count, uint32_t *bins,
                     uint32_t *rm, int cus, hipStream_t s)
{
    const bool paired = W <= 8 && a.e_pair == nullptr && a.e_uniform <= 7u;
    const bool use_rm = rm != nullptr && !paired;
    const uint32_t rm_stride = (a.rows + 3u) & ~3u;
    int per_cu = 1, per_cu1 = 1;
    hipError_t oe = use_rm ? verify_blocks_per_cu<W, L, false, true>(per_cu1)
                           : verify_blocks_per_cu<W, L, false>(per_cu1);
    if (oe == hipSuccess && paired)
        oe = verify_blocks_per_cu<W, L, true>(per_cu);
    if (oe != hipSuccess)
        return oe;
    if (use_rm && a.n_reads > 0) {
        hipLaunchKernelGGL(k_reads_rowmajor, dim3((a.n_reads + 255u) / 256u), dim3(256),
                           (size_t)256u * (rm_stride + 1u) * 4u, s, a.reads, a.pitch, a.rows,
                           a.n_reads, rm_stride, rm);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    const uint64_t CHUNK = 1ull << 30;
    for (uint64_t first = 0; first < a.n_pairs; first += CHUNK) {
        FilterArgs c = a;
        const uint64_t n = a.n_pairs - first < CHUNK ? a.n_pairs - first : CHUNK;
        c.n_pairs = n;
        c.pair_read = a.pair_read ? a.pair_read + first : nullptr;
        if (!a.pair_read && first > 0)
            c.n_reads = 0;   // pair i uses read i < n_reads < 2^30: none here
        c.cand_pos = a.cand_pos + first;
        c.e_pair = a.e_pair ? a.e_pair + first : nullptr;
        c.accept = nullptr;
        c.est = nullptr;
        c.accept_bits = nullptr;
        const uint8_t *acc = accept ? accept + first : nullptr;
        uint16_t *out = dist + first;
        const uint64_t want = (n + 255) / 256;
        const uint32_t groups = (uint32_t)((n + SEL_PER_GROUP - 1) / SEL_PER_GROUP);
        const bool vec = ((uintptr_t)acc & 15u) == 0 && ((uintptr_t)out & 15u) == 0;
        if (c.e_pair) {
            // per-pair e: listed by (length in words, e) over the whole batch
            hipLaunchKernelGGL(k_bin_zero, dim3(32), dim3(256), 0, s, bins);
            if (vec)
                hipLaunchKernelGGL(k_bin_count<true>, dim3(groups), dim3(256), 0, s, c, acc,
                                   (uint32_t)n, bins, out);
            else
                hipLaunchKernelGGL(k_bin_count<false>, dim3(groups), dim3(256), 0, s, c, acc,
                                   (uint32_t)n, bins, out);
            hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, s, bins, count);
            if (vec)
                hipLaunchKernelGGL(k_bin_write<true>, dim3(groups), dim3(256), 0, s, c, acc,
                                   (uint32_t)n, bins, list);
            else
                hipLaunchKernelGGL(k_bin_write<false>, dim3(groups), dim3(256), 0, s, c, acc,
                                   (uint32_t)n, bins, list);
        } else {
            if (vec)
                hipLaunchKernelGGL(k_select_count<true>, dim3(groups), dim3(256), 0, s, acc,
                                   (uint32_t)n, groups_buf, out);
            else
                hipLaunchKernelGGL(k_select_count<false>, dim3(groups), dim3(256), 0, s, acc,
                                   (uint32_t)n, groups_buf, out);
            hipLaunchKernelGGL(k_select_scan, dim3(1), dim3(1024), 0, s, groups_buf, groups,
                               count);
            if (vec)
                hipLaunchKernelGGL(k_select_write<true>, dim3(groups), dim3(256), 0, s, c, acc,
                                   (uint32_t)n, groups_buf, list);
            else
                hipLaunchKernelGGL(k_select_write<false>, dim3(groups), dim3(256), 0, s, c, acc,
                                   (uint32_t)n, groups_buf, list);
        }
        // Grids of up to 8 times the resident workgroups: later workgroups
        // start as earlier ones finish, so the waves' gathers do not all come
        // at once (measured faster than one resident round at every sweep
        // point; the list length is only known on the device).
        const uint64_t vb1 = want < 8ull * cus * per_cu1 ? want : 8ull * cus * per_cu1;
        if (paired) {
            const uint64_t want2 = (n + 511) / 512;        // two pairs per lane
            const uint64_t vb = want2 < 8ull * cus * per_cu ? want2 : 8ull * cus * per_cu;
            hipLaunchKernelGGL((k_verify_paired<W, L>), dim3((uint32_t)vb), dim3(256), 0, s, c,
                               list, count, out, deferred, count + 1);
            // the waves it could not pair (count[1] entries, usually none:
            // one resident round)
            const uint64_t vbd = want < (uint64_t)cus * per_cu1 ? want : (uint64_t)cus * per_cu1;
            hipLaunchKernelGGL((k_verify<W, L>), dim3((uint32_t)vbd), dim3(256), 0, s, c,
                               (const uint32_t *)deferred, (const uint32_t *)(count + 1), out,
                               (const uint32_t *)nullptr, 0u);
        } else if (use_rm) {
            hipLaunchKernelGGL((k_verify<W, L, true>), dim3((uint32_t)vb1), dim3(256), 0, s, c,
                               list, count, out, (const uint32_t *)rm, rm_stride);
        } else {
            hipLaunchKernelGGL((k_verify<W, L>), dim3((uint32_t)vb1), dim3(256), 0, s, c, list,
                               count, out, (const uint32_t *)nullptr, 0u);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

template <int L>
hipError_t verify_l(const FilterArgs &a, const uint8_t *accept, uint16_t *dist, uint32_t *list,
                    uint32_t *groups_buf, uint32_t *deferred, uint32_t *count, uint32_t *bins,
                    uint32_t *rm, uint32_t words, int cus, hipStream_t s)
{
    switch (words) {
    case 1: return verify_wl<1, L>(a, accept, dist, list, groups_buf, deferred, count, bins, rm, cus,
                                  s);
    case 2: return verify_wl<2, L>(a, accept, dist, list, groups_buf, deferred, count, bins, rm, cus,
                                  s);
    case 3: return verify_wl<3, L>(a, accept, dist, list, groups_buf, deferred, count, bins, rm, cus,
                                  s);
    case 4: return verify_wl<4, L>(a, accept, dist, list, groups_buf, deferred, count, bins, rm, cus,
                                  s);
    case 5: return verify_wl<5, L>(a, accept, dist, list, groups_buf, deferred, count, bins, rm, cus,
                                  s);
    case 6: return verify_wl<6, L>(a, accept, dist, list, groups_buf, deferred, count, bins, rm, cus,
                                  s);
    case 7: return verify_wl<7, L>(a, accept, dist, list, groups_buf, deferred, count, bins, rm, cus,
                                  s);
    case 8: return verify_wl<8, L>(a, accept, dist, list, groups_buf, deferred, count, bins, rm, cus,
                                  s);
    case 9: return verify_wl<9, L>(a, accept, dist, list, groups_buf, deferred, count, bins, rm, cus,
                                  s);
    case 10: return verify_wl<10, L>(a, accept, dist, list, groups_buf, deferred, count, bins, rm, cus,
                                  s);
    case 11: return verify_wl<11, L>(a, accept, dist, list, groups_buf, deferred, count, bins, rm, cus,
                                  s);
    case 12: return verify_wl<12, L>(a, accept, dist, list, groups_buf, deferred, count, bins, rm, cus,
                                  s);
    case 13: return verify_wl<13, L>(a, accept, dist, list, groups_buf, deferred, count, bins, rm, cus,
                                  s);
    case 14: return verify_wl<14, L>(a, accept, dist, list, groups_buf, deferred, count, bins, rm, cus,
                                  s);
    case 15: return verify_wl<15, L>(a, accept, dist, list, groups_buf, deferred, count, bins, rm, cus,
                                  s);
    case 16: return verify_wl<16, L>(a, accept, dist, list, groups_buf, deferred, count, bins, rm, cus,
                                  s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_verify(const FilterArgs &a, const uint8_t *accept, uint16_t *dist,
                         uint32_t *list, uint32_t *groups, uint32_t *deferred, uint32_t *count,
                         uint32_t *bins, uint32_t *reads_rm, uint32_t words, uint32_t layout,
                         int cus, hipStream_t s)
{
    return layout == GK_READS_INTERLEAVED
               ? verify_l<GK_READS_INTERLEAVED>(a, accept, dist, list, groups, deferred, count,
                                                bins, reads_rm, words, cus, s)
               : verify_l<GK_READS_SPLIT>(a, accept, dist, list, groups, deferred, count, bins,
                                          reads_rm, words, cus, s);
}

}  // namespace gkd

// Plain GateKeeper-GPU filter launch for gfx950: one lane per pair (the
// per-pair body is in gk_pair.h), over a grid-stride loop.
//
// Two shapes, chosen by GK_OPT_PAIRS_PER_LANE (results are identical):
//   k_filter_single  one pair per lane, the whole batch in one grid;
//   k_filter         a smaller grid whose lanes walk several pairs, keeping two
//                    pairs' loads in flight ahead of the one being computed
//                    (the next pair's read and window words, the indices of the
//                    pair after).  Those loads use clamped indices, so no
//                    branch surrounds them; the tail reloads the last pair.
#include "gk_pair.h"

namespace gkd {
namespace {

// One pair per lane, no loop: the smallest register footprint (the most
// waves per SIMD to hide the gather latency).
template <int W, int L, bool VAR = false>
__global__ __launch_bounds__(256) void k_filter_single(FilterArgs a)
{
    const uint32_t n = (uint32_t)a.n_pairs;
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    uint32_t res = GK_INVALID;
    if (i < n) {
        const PairIdx p = load_idx(a, i);
        PairData<W> d;
        load_data<W>(a, p, d);
        uint32_t est;
        res = compute_pair<W, L, true, VAR>(a, p, d, est);
        __builtin_nontemporal_store((uint8_t)res, a.accept + i);
        __builtin_nontemporal_store((uint16_t)est, a.est + i);
    }
    if (a.accept_bits) {
        const unsigned long long bits = __ballot(i < n && (res == GK_ACCEPT || res == GK_UNDEFINED));
        if ((threadIdx.x & 63u) == 0u && i < n)
            a.accept_bits[i >> 6] = bits;
    }
}

template <int W, int L>
__global__ __launch_bounds__(256) void k_filter(FilterArgs a)
{
    const uint32_t n = (uint32_t)a.n_pairs;   // < 2^30 per launch (host splits)
    const uint32_t stride = gridDim.x * 256u;
    uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= n)
        return;

    // Buffers A and B alternate between "computing" and "in flight", so the
    // loop carries no copies of the data registers.
    PairIdx ia = load_idx(a, i);
    PairData<W> da, db;
    load_data<W>(a, ia, da);
    PairIdx ib = load_idx(a, min(i + stride, n - 1));

    while (true) {
        {
            load_data<W>(a, ib, db);
            const PairIdx in = load_idx(a, min(i + 2 * stride, n - 1));
            uint32_t est;
            const uint32_t res = compute_pair<W, L>(a, ia, da, est);
            __builtin_nontemporal_store((uint8_t)res, a.accept + i);
            __builtin_nontemporal_store((uint16_t)est, a.est + i);
            if (a.accept_bits) {
                const unsigned long long bits = __ballot(res == GK_ACCEPT || res == GK_UNDEFINED);
                if ((threadIdx.x & 63u) == 0u)
                    a.accept_bits[i >> 6] = bits;
            }
            ia = in;
            i += stride;
            if (i >= n)
                break;
        }
        {
            load_data<W>(a, ia, da);
            const PairIdx in = load_idx(a, min(i + 2 * stride, n - 1));
            uint32_t est;
            const uint32_t res = compute_pair<W, L>(a, ib, db, est);
            __builtin_nontemporal_store((uint8_t)res, a.accept + i);
            __builtin_nontemporal_store((uint16_t)est, a.est + i);
            if (a.accept_bits) {
                const unsigned long long bits = __ballot(res == GK_ACCEPT || res == GK_UNDEFINED);
                if ((threadIdx.x & 63u) == 0u)
                    a.accept_bits[i >> 6] = bits;
            }
            ib = in;
            i += stride;
            if (i >= n)
                break;
        }
    }
}

template <int W, int L>
hipError_t launch_wl(const FilterArgs &a, uint32_t pairs_per_lane, hipStream_t s)
{
    static int max_blocks = -1;   // resident 256-lane blocks on the whole device
    if (max_blocks < 0) {
        int dev = 0, cus = 0, per_cu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_filter<W, L>, 256, 0);
        if (e != hipSuccess)
            return e;
        max_blocks = cus * (per_cu > 0 ? per_cu : 1);
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
        c.accept = a.accept + first;
        c.est = a.est + first;
        c.accept_bits = a.accept_bits ? a.accept_bits + first / 64 : nullptr;
        const uint64_t full = (n + 255) / 256;
        uint64_t blocks = full;
        if (a.flags != 0u) {
            // Variant semantics: their own one-pair-per-lane kernel, so the
            // default kernels carry no variant code.
            hipLaunchKernelGGL((k_filter_single<W, L, true>), dim3((uint32_t)full), dim3(256), 0,
                               s, c);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess)
                return e;
            continue;
        }
        if (pairs_per_lane == 0) {
            // Automatic: one pair per lane.  Measured over 100 bp at e = 0..10
            // and 150 / 250 bp at 2-10 % thresholds, it beat four pairs per
            // lane (each lane prefetching its next pair) at every point, light
            // pairs (gather-bound) and heavy ones (VALU-bound) alike.
            pairs_per_lane = 1u;
        }
        if (pairs_per_lane == 1) {
            hipLaunchKernelGGL((k_filter_single<W, L>), dim3((uint32_t)full), dim3(256), 0, s, c);
        } else {
            const uint64_t want = (n + 256ull * pairs_per_lane - 1) / (256ull * pairs_per_lane);
            blocks = want < 1 ? 1 : want;
            if (pairs_per_lane == GK_PPL_RESIDENT && blocks > (uint64_t)max_blocks)
                blocks = max_blocks;          // exactly one residency of the device
            hipLaunchKernelGGL((k_filter<W, L>), dim3((uint32_t)blocks), dim3(256), 0, s, c);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

template <int L>
hipError_t launch_l(const FilterArgs &a, uint32_t words, uint32_t ppl, hipStream_t s)
{
    switch (words) {
    case 1: return launch_wl<1, L>(a, ppl, s);
    case 2: return launch_wl<2, L>(a, ppl, s);
    case 3: return launch_wl<3, L>(a, ppl, s);
    case 4: return launch_wl<4, L>(a, ppl, s);
    case 5: return launch_wl<5, L>(a, ppl, s);
    case 6: return launch_wl<6, L>(a, ppl, s);
    case 7: return launch_wl<7, L>(a, ppl, s);
    case 8: return launch_wl<8, L>(a, ppl, s);
    case 9: return launch_wl<9, L>(a, ppl, s);
    case 10: return launch_wl<10, L>(a, ppl, s);
    case 11: return launch_wl<11, L>(a, ppl, s);
    case 12: return launch_wl<12, L>(a, ppl, s);
    case 13: return launch_wl<13, L>(a, ppl, s);
    case 14: return launch_wl<14, L>(a, ppl, s);
    case 15: return launch_wl<15, L>(a, ppl, s);
    case 16: return launch_wl<16, L>(a, ppl, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_filter(const FilterArgs &a, uint32_t words, uint32_t layout,
                         uint32_t pairs_per_lane, hipStream_t s)
{
    return layout == GK_READS_INTERLEAVED
               ? launch_l<GK_READS_INTERLEAVED>(a, words, pairs_per_lane, s)
               : launch_l<GK_READS_SPLIT>(a, words, pairs_per_lane, s);
}

}  // namespace gkd

// Mixed-batch GateKeeper-GPU filter for gfx950: one persistent launch over a
// batch whose pairs differ in read length and threshold.
//
// The paper fixes the read length and e at compile time (Sec. 3.1, 3.2) and
// so runs one kernel per (length, e) group.  Here one persistent grid takes
// the whole batch:
//   - each workgroup repeatedly claims a tile of T consecutive pairs from a
//     device counter;
//   - it classifies the tile's pairs (invalid and undefined pairs are written
//     at once, pairs with more than 31 shifts go to a residual list) and
//     counting-sorts the rest in LDS by (words per mask W, k_max), so that a
//     64-lane chunk holds one W and nearly equal e;
//   - its waves take chunks from an LDS counter and run the register-only
//     fast path of gk_pair.h for the chunk's W (a wave-uniform switch), one
//     or two pairs per lane (two: both pairs' loads in flight before either
//     is computed; only for up to 10 words per mask, where the registers for
//     it fit); results go back to the pairs' own slots.
// Residual pairs are filtered afterwards by the general path, and the accept
// bits (if wanted) by a pass over the accept codes.  The host captures the
// four launches in one hipGraph.
#include "gk_pair.h"

namespace gkd {

namespace {

constexpr uint32_t NBINS = 16 * 32;       // W in 1..16, k_max in 0..31
constexpr uint32_t KEY_DONE = 0xFFFFu;

struct MixedLds {
    uint32_t hist[NBINS];
    uint32_t wstart[17];
    uint32_t tile;
    uint32_t n_chunks;
    uint32_t next_chunk;
};

// Dynamic LDS after MixedLds: keys[T] u16, sorted[T] u16, chunk_start[C] u32,
// chunk_info[C] u32 with C = T/64 + 16, then the tile's results out_est[T] u16
// and out_acc[T] u8, written back to HBM in slot order once the tile is done
// (results land in sorted order, so writing them directly would scatter
// partial-line writes).
__host__ __device__ inline uint32_t mixed_chunk_cap(uint32_t tile) { return tile / 64 + 16; }

__host__ inline size_t mixed_lds_bytes(uint32_t tile)
{
    return sizeof(MixedLds) + 2u * tile * sizeof(uint16_t) + 2u * mixed_chunk_cap(tile) * 4u +
           3u * tile;
}

struct TileOut {
    uint8_t *acc;
    uint16_t *est;
};

template <int W, int L, bool VAR>
__device__ __forceinline__ void run_chunk_pair(const FilterArgs &a, const TileOut &o,
                                               uint32_t base, uint32_t slot)
{
    const PairIdx p = load_idx(a, base + slot);
    PairData<W> d;
    load_data<W>(a, p, d);
    uint32_t est;
    const uint32_t res = compute_pair<W, L, false, VAR>(a, p, d, est);
    o.acc[slot] = (uint8_t)res;
    o.est[slot] = (uint16_t)est;
}

template <int W, int L, bool VAR>
__device__ __forceinline__ void run_chunk_pair2(const FilterArgs &a, const TileOut &o,
                                                uint32_t base, uint32_t s0, bool has1,
                                                uint32_t s1)
{
    // both pairs' loads in flight before either is computed
    const PairIdx p0 = load_idx(a, base + s0);
    const PairIdx p1 = load_idx(a, base + (has1 ? s1 : s0));
    PairData<W> d0, d1;
    load_data<W>(a, p0, d0);
    load_data<W>(a, p1, d1);
    uint32_t est;
    uint32_t res = compute_pair<W, L, false, VAR>(a, p0, d0, est);
    o.acc[s0] = (uint8_t)res;
    o.est[s0] = (uint16_t)est;
    if (has1) {
        res = compute_pair<W, L, false, VAR>(a, p1, d1, est);
        o.acc[s1] = (uint8_t)res;
        o.est[s1] = (uint16_t)est;
    }
}

template <int WMAX, int L, int PPL, bool VAR>
__device__ __forceinline__ void run_chunk(const FilterArgs &a, const TileOut &o, uint32_t base,
                                          uint32_t w, uint32_t s0, bool has1, uint32_t s1)
{
#define GK_CASE(N)                                                                 \
    case N:                                                                        \
        if (N <= WMAX) {                                                           \
            if (PPL == 2)                                                          \
                run_chunk_pair2<(N <= WMAX ? N : 1), L, VAR>(a, o, base, s0, has1, s1); \
            else                                                                   \
                run_chunk_pair<(N <= WMAX ? N : 1), L, VAR>(a, o, base, s0);       \
        }                                                                          \
        break;
    switch (w) {
        GK_CASE(1) GK_CASE(2) GK_CASE(3) GK_CASE(4) GK_CASE(5) GK_CASE(6) GK_CASE(7) GK_CASE(8)
        GK_CASE(9) GK_CASE(10) GK_CASE(11) GK_CASE(12) GK_CASE(13) GK_CASE(14) GK_CASE(15)
        GK_CASE(16)
    default:
        break;
    }
#undef GK_CASE
}

// Batch of a tile in a table launch: the last b with prefix[b] <= tile (empty
// batches share their prefix with the next one, so the last match is the
// batch that owns the tile).
__device__ __forceinline__ uint32_t table_batch(const BatchTable *t, uint32_t tile)
{
    uint32_t lo = 0, hi = t->n_batches;          // prefix[hi] > tile
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (t->prefix[mid] <= tile)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

template <int WMAX, int L, int PPL, bool VAR = false>
__global__ __launch_bounds__(256) void k_mixed(FilterArgs a0, MixedArgs x)
{
    extern __shared__ uint32_t lds_raw[];
    MixedLds &s = *reinterpret_cast<MixedLds *>(lds_raw);
    uint16_t *keys = reinterpret_cast<uint16_t *>(lds_raw + sizeof(MixedLds) / 4);
    uint16_t *sorted = keys + x.tile;
    uint32_t *chunk_start = reinterpret_cast<uint32_t *>(sorted + x.tile);
    uint32_t *chunk_info = chunk_start + mixed_chunk_cap(x.tile);
    TileOut out;
    out.est = reinterpret_cast<uint16_t *>(chunk_info + mixed_chunk_cap(x.tile));
    out.acc = reinterpret_cast<uint8_t *>(out.est + x.tile);

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u;
    const uint32_t n_tiles = x.table ? x.table->prefix[x.table->n_batches] : x.n_tiles;

    while (true) {
        if (tid == 0)
            s.tile = atomicAdd(x.tile_counter, 1u);
        for (uint32_t b = tid; b < NBINS; b += 256)
            s.hist[b] = 0;
        __syncthreads();
        const uint32_t tile = s.tile;
        if (tile >= n_tiles)
            break;
        // Residual entries are launch-wide ids tile * T + slot.
        const uint32_t gbase = tile * x.tile;
        FilterArgs a = a0;
        uint32_t base = gbase;
        if (x.table) {
            const uint32_t b = table_batch(x.table, tile);
            a = x.table->args[b];
            base = (tile - x.table->prefix[b]) * x.tile;
        }
        const uint32_t n = (uint32_t)a.n_pairs;

        // 1. classify
        for (uint32_t j = tid; j < x.tile; j += 256) {
            const uint32_t i = base + j;
            uint32_t key = KEY_DONE;
            if (i < n) {
                const PairIdx p = load_idx(a, i);
                const uint32_t m = p.r < a.n_reads ? (uint32_t)a.read_len[p.r] : 0u;
                if (m == 0u || m > a.max_read_len) {
                    out.acc[j] = GK_INVALID;
                    out.est[j] = GK_EST_NONE;
                } else if ((uint64_t)p.pos + m > a.ref_len ||
                           (a.read_has_n && a.read_has_n[p.r])) {
                    out.acc[j] = GK_UNDEFINED;
                    out.est[j] = GK_EST_NONE;
                } else {
                    const uint32_t kmax = p.e < m - 1u ? p.e : m - 1u;
                    const uint32_t w = (m + 31u) / 32u;
                    if (kmax > 31u || w > (uint32_t)WMAX) {
                        x.resid_list[atomicAdd(x.resid_count, 1u)] = gbase + j;
                    } else {
                        key = (w - 1u) * 32u + (x.sort_e ? kmax : 0u);
                        atomicAdd(&s.hist[key], 1u);
                    }
                }
            }
            keys[j] = (uint16_t)key;
        }
        __syncthreads();

        // 2. exclusive prefix over the bins (wave 0: 8 bins per lane)
        if (tid < 64) {
            uint32_t local[8], sum = 0;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                local[q] = s.hist[tid * 8 + q];
                sum += local[q];
            }
            uint32_t incl = sum;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t v = __shfl_up(incl, o, 64);
                if (lane >= (uint32_t)o)
                    incl += v;
            }
            uint32_t run = incl - sum;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint32_t b = tid * 8 + q;
                if (b % 32u == 0u)
                    s.wstart[b / 32u] = run;
                s.hist[b] = run;
                run += local[q];
            }
            if (tid == 63)
                s.wstart[16] = run;
        }
        __syncthreads();

        // 3. scatter slots into bin order
        for (uint32_t j = tid; j < x.tile; j += 256) {
            const uint32_t key = keys[j];
            if (key != KEY_DONE)
                sorted[atomicAdd(&s.hist[key], 1u)] = (uint16_t)j;
        }

        // 4. chunks: runs of one W, 64 * ppl pairs at most.  A W's pairs are
        //    in ascending k_max, so its one partial chunk is put first, on the
        //    pairs with the fewest shifts: its idle lanes then wait through
        //    the shortest loop.
        if (tid < 64) {
            const uint32_t ch = 64u * PPL;
            const uint32_t w0 = tid < 16 ? s.wstart[tid] : 0u;
            const uint32_t cnt = tid < 16 ? s.wstart[tid + 1] - w0 : 0u;
            const uint32_t nch = (cnt + ch - 1) / ch;
            const uint32_t lead = cnt % ch == 0u ? ch : cnt % ch;   // size of chunk 0
            uint32_t incl = nch;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t v = __shfl_up(incl, o, 64);
                if (lane >= (uint32_t)o)
                    incl += v;
            }
            const uint32_t first = incl - nch;
            for (uint32_t c = 0; c < nch; ++c) {
                chunk_start[first + c] = w0 + (c == 0u ? 0u : lead + (c - 1u) * ch);
                chunk_info[first + c] = (c == 0u ? lead : ch) | ((tid + 1u) << 16);
            }
            if (tid == 63) {
                s.n_chunks = incl;
                s.next_chunk = 0;
            }
        }
        __syncthreads();

        // 5. waves take chunks, the heaviest (largest W and k_max, at the
        //    end of the list) first, so the tile ends on short chunks
        const uint32_t n_chunks = s.n_chunks;
        while (true) {
            uint32_t c = 0;
            if (lane == 0)
                c = atomicAdd(&s.next_chunk, 1u);
            c = __shfl(c, 0, 64);
            if (c >= n_chunks)
                break;
            c = n_chunks - 1u - c;
            const uint32_t start = chunk_start[c];
            const uint32_t info = chunk_info[c];
            const uint32_t cnt = info & 0xFFFFu;
            const uint32_t w = __builtin_amdgcn_readfirstlane(info >> 16);
            if (lane < cnt) {
                const uint32_t s0 = sorted[start + lane];
                const bool has1 = lane + 64u < cnt;
                const uint32_t s1 = has1 ? sorted[start + lane + 64u] : s0;
                run_chunk<WMAX, L, PPL, VAR>(a, out, base, w, s0, has1, s1);
            }
        }
        __syncthreads();

        // 6. write the tile's results back in slot order (residual pairs'
        //    slots hold placeholders; the residual pass overwrites them later)
        const uint32_t live = n - base < x.tile ? n - base : x.tile;
        for (uint32_t j = tid; j < live; j += 256) {
            a.accept[base + j] = out.acc[j];
            a.est[base + j] = out.est[j];
        }
        __syncthreads();
    }
}

template <int W, int L, bool VAR = false>
__global__ __launch_bounds__(256) void k_residual(FilterArgs a0, const BatchTable *table,
                                                  uint32_t tile_size, const uint32_t *list,
                                                  const uint32_t *count)
{
    const uint32_t total = *count;
    for (uint32_t j = blockIdx.x * 256u + threadIdx.x; j < total; j += gridDim.x * 256u) {
        uint32_t i = list[j];
        FilterArgs a = a0;
        if (table) {
            const uint32_t tile = i / tile_size;
            const uint32_t b = table_batch(table, tile);
            a = table->args[b];
            i -= table->prefix[b] * tile_size;
        }
        const PairIdx p = load_idx(a, i);
        PairData<W> d;
        load_data<W>(a, p, d);
        uint32_t est;
        const uint32_t res = compute_pair<W, L, true, VAR>(a, p, d, est);
        a.accept[i] = (uint8_t)res;
        a.est[i] = (uint16_t)est;
    }
}

__global__ __launch_bounds__(256) void k_reset(uint32_t *tile_counter, uint32_t *resid_count)
{
    if (threadIdx.x == 0) {
        *tile_counter = 0;
        *resid_count = 0;
    }
}

// One thread per 64 pairs: bit j of word t = pair 64t+j is ACCEPT or UNDEFINED.
__global__ __launch_bounds__(256) void k_accept_bits(const uint8_t *accept, uint64_t n,
                                                     unsigned long long *bits)
{
    const uint64_t t = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    if (t * 64 >= n)
        return;
    unsigned long long word = 0;
    const uint64_t first = t * 64;
    const uint32_t cnt = (uint32_t)(n - first < 64 ? n - first : 64);
    for (uint32_t j = 0; j < cnt; ++j) {
        const uint32_t v = accept[first + j];
        word |= (unsigned long long)(v == GK_ACCEPT || v == GK_UNDEFINED) << j;
    }
    bits[t] = word;
}

template <int WMAX, int L>
hipError_t launch_mixed_wl(const FilterArgs &a, const MixedArgs &x0, hipStream_t s)
{
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
        c.accept_bits = nullptr;
        MixedArgs x = x0;
        x.n_tiles = (uint32_t)((n + x.tile - 1) / x.tile);
        hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, x.tile_counter, x.resid_count);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        const uint32_t blocks = x.blocks < x.n_tiles ? x.blocks : x.n_tiles;
        if (c.flags != 0u) {
            // Variant semantics: their own kernels, one pair per lane.
            hipLaunchKernelGGL((k_mixed<WMAX, L, 1, true>), dim3(blocks), dim3(256),
                               mixed_lds_bytes(x.tile), s, c, x);
            if ((e = hipGetLastError()) != hipSuccess)
                return e;
            hipLaunchKernelGGL((k_residual<WMAX, L, true>), dim3(x.resid_blocks), dim3(256), 0,
                               s, c, (const BatchTable *)nullptr, x.tile,
                               (const uint32_t *)x.resid_list, (const uint32_t *)x.resid_count);
        } else if constexpr (WMAX <= 10) {
            if (x.ppl == 2)
                hipLaunchKernelGGL((k_mixed<WMAX, L, 2>), dim3(blocks), dim3(256),
                                   mixed_lds_bytes(x.tile), s, c, x);
            else
                hipLaunchKernelGGL((k_mixed<WMAX, L, 1>), dim3(blocks), dim3(256),
                                   mixed_lds_bytes(x.tile), s, c, x);
        } else {
            hipLaunchKernelGGL((k_mixed<WMAX, L, 1>), dim3(blocks), dim3(256),
                               mixed_lds_bytes(x.tile), s, c, x);
        }
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        if (c.flags == 0u)
            hipLaunchKernelGGL((k_residual<WMAX, L>), dim3(x.resid_blocks), dim3(256), 0, s, c,
                               (const BatchTable *)nullptr, x.tile,
                               (const uint32_t *)x.resid_list, (const uint32_t *)x.resid_count);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        if (a.accept_bits) {
            const uint64_t words = (n + 63) / 64;
            hipLaunchKernelGGL(k_accept_bits, dim3((uint32_t)((words + 255) / 256)), dim3(256), 0,
                               s, (const uint8_t *)c.accept, n, a.accept_bits + first / 64);
            if ((e = hipGetLastError()) != hipSuccess)
                return e;
        }
    }
    return hipSuccess;
}

template <int WMAX, int L>
hipError_t launch_table_wl(const MixedArgs &x, hipStream_t s)
{
    FilterArgs none{};
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, x.tile_counter, x.resid_count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if constexpr (WMAX <= 10) {
        if (x.ppl == 2)
            hipLaunchKernelGGL((k_mixed<WMAX, L, 2>), dim3(x.blocks), dim3(256),
                               mixed_lds_bytes(x.tile), s, none, x);
        else
            hipLaunchKernelGGL((k_mixed<WMAX, L, 1>), dim3(x.blocks), dim3(256),
                               mixed_lds_bytes(x.tile), s, none, x);
    } else {
        hipLaunchKernelGGL((k_mixed<WMAX, L, 1>), dim3(x.blocks), dim3(256),
                           mixed_lds_bytes(x.tile), s, none, x);
    }
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    hipLaunchKernelGGL((k_residual<WMAX, L>), dim3(x.resid_blocks), dim3(256), 0, s, none,
                       x.table, x.tile, (const uint32_t *)x.resid_list,
                       (const uint32_t *)x.resid_count);
    return hipGetLastError();
}

template <int L>
hipError_t launch_mixed_l(const FilterArgs &a, const MixedArgs &x, uint32_t wmax, hipStream_t s)
{
    if (wmax <= 4)
        return launch_mixed_wl<4, L>(a, x, s);
    if (wmax <= 10)
        return launch_mixed_wl<10, L>(a, x, s);
    return launch_mixed_wl<16, L>(a, x, s);
}

template <int WMAX, int L>
hipError_t occupancy_wl(uint32_t tile, uint32_t ppl, int *blocks_per_cu)
{
    if constexpr (WMAX <= 10) {
        if (ppl == 2)
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                blocks_per_cu, k_mixed<WMAX, L, 2>, 256, mixed_lds_bytes(tile));
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_mixed<WMAX, L, 1>, 256,
                                                        mixed_lds_bytes(tile));
}

}  // namespace

size_t mixed_lds_size(uint32_t tile) { return mixed_lds_bytes(tile); }

hipError_t mixed_blocks_per_cu(uint32_t wmax, uint32_t layout, uint32_t tile, uint32_t ppl,
                               int *out)
{
    const bool il = layout == GK_READS_INTERLEAVED;
    if (wmax <= 4)
        return il ? occupancy_wl<4, GK_READS_INTERLEAVED>(tile, ppl, out)
                  : occupancy_wl<4, GK_READS_SPLIT>(tile, ppl, out);
    if (wmax <= 10)
        return il ? occupancy_wl<10, GK_READS_INTERLEAVED>(tile, ppl, out)
                  : occupancy_wl<10, GK_READS_SPLIT>(tile, ppl, out);
    return il ? occupancy_wl<16, GK_READS_INTERLEAVED>(tile, ppl, out)
              : occupancy_wl<16, GK_READS_SPLIT>(tile, ppl, out);
}

hipError_t launch_mixed_table(const MixedArgs &x, uint32_t wmax, uint32_t layout, hipStream_t s)
{
    const bool il = layout == GK_READS_INTERLEAVED;
    if (wmax <= 4)
        return il ? launch_table_wl<4, GK_READS_INTERLEAVED>(x, s)
                  : launch_table_wl<4, GK_READS_SPLIT>(x, s);
    if (wmax <= 10)
        return il ? launch_table_wl<10, GK_READS_INTERLEAVED>(x, s)
                  : launch_table_wl<10, GK_READS_SPLIT>(x, s);
    return il ? launch_table_wl<16, GK_READS_INTERLEAVED>(x, s)
              : launch_table_wl<16, GK_READS_SPLIT>(x, s);
}

hipError_t launch_accept_bits(const uint8_t *accept, uint64_t n, unsigned long long *bits,
                              hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    const uint64_t words = (n + 63) / 64;
    hipLaunchKernelGGL(k_accept_bits, dim3((uint32_t)((words + 255) / 256)), dim3(256), 0, s,
                       accept, n, bits);
    return hipGetLastError();
}

hipError_t launch_mixed(const FilterArgs &a, const MixedArgs &x, uint32_t wmax, uint32_t layout,
                        hipStream_t s)
{
    return layout == GK_READS_INTERLEAVED
               ? launch_mixed_l<GK_READS_INTERLEAVED>(a, x, wmax, s)
               : launch_mixed_l<GK_READS_SPLIT>(a, x, wmax, s);
}

}  // namespace gkd

// The filter with its reads encoded in the same launch: the paper's kernel
// encodes the sequences itself when they reach it in ASCII (Sec. 3.3), the
// device-encoded mode of its throughput tables (Sec. 5.2, Table 2).  Pair i
// compares read i with its window.
//
// A workgroup takes 256 consecutive pairs, whose reads' text is one
// contiguous span.  It stages the span as three bit-planes in LDS (low code
// bits, high code bits, unknown bases), as the staged read encoder does, and
// each lane cuts its read's 16-base words out of the planes with funnel
// shifts straight into registers: the encoded reads never go to memory, and
// the launch reads each text byte once.  A read outside the staged span
// (offsets out of order, or a read longer than the rows hold) is encoded from
// global memory by its own lane.  From there on a pair is filtered exactly as
// by the plain launch.
#include "gk_encode_dev.h"
#include "gk_internal.h"
#include "gk_pair.h"

namespace gkd {
namespace {

// Split-layout words (low code bits in bits 0-15, high in 16-31) of 16 bases
// starting at byte `first` of a read at `off`, from global memory; sets
// `unknown` if a byte other than A/C/G/T is among them.
__device__ __forceinline__ uint32_t word_direct(const uint8_t *ascii, uint64_t off, uint64_t len,
                                                uint64_t first, uint32_t &unknown)
{
    if (first >= len)
        return 0u;
    const uint32_t n = (uint32_t)((len - first) < 16 ? (len - first) : 16);
    uint32_t b[4];
    load16(ascii + off + first, n, b);
    uint32_t word = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const uint32_t c = (b[j >> 2] >> (8 * (j & 3))) & 0xFFu;
        if ((uint32_t)j < n) {
            const uint32_t code = code_of(c);
            word |= ((code & 1u) << j) | ((code >> 1) << (16 + j));
            unknown |= is_base(c) ? 0u : 1u;
        }
    }
    return word;
}

// Up to 4 words per mask (reads of 128 bases) the paper's filter fits in 64
// registers, so eight waves per SIMD.
template <int W, bool VAR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W <= 4 && !VAR ? 8 : 1)))
void k_filter_ascii(FilterArgs a, const uint8_t *ascii,
                                                      const uint64_t *read_off)
{
    extern __shared__ uint32_t fa_lds[];
    const uint32_t rows = a.rows;
    const uint32_t cap = enc_cap_words(rows);
    uint32_t *p_lo = fa_lds;
    uint32_t *p_hi = fa_lds + (cap + 1u);
    uint32_t *p_un = fa_lds + 2u * (cap + 1u);

    const uint32_t n = (uint32_t)a.n_pairs;
    const uint32_t r0 = blockIdx.x * ENC_G;
    const uint32_t r1 = n - r0 < ENC_G ? n : r0 + ENC_G;
    const uint64_t base = read_off[r0];
    const uint64_t end = read_off[r1];
    const uint64_t a0 = base & ~31ull;                  // span start, 32-byte aligned
    const bool staged = end >= base && end - a0 <= 32ull * cap;
    uint32_t nw = 0;
    if (staged) {
        nw = (uint32_t)((end - a0 + 31u) / 32u);
        for (uint32_t j = threadIdx.x; j < nw; j += 256u) {
            const uint64_t at = a0 + 32ull * j;
            const uint32_t cnt = end - at < 32u ? (uint32_t)(end - at) : 32u;
            uint32_t d[8];
            load_chunk(ascii + at, cnt, d);
            uint32_t lo, hi, un;
            chunk_planes(d, cnt, lo, hi, un);
            p_lo[j] = lo;
            p_hi[j] = hi;
            p_un[j] = un;
        }
        if (threadIdx.x == 0) {
            p_lo[nw] = 0u;
            p_hi[nw] = 0u;
            p_un[nw] = 0u;
        }
    }
    __syncthreads();

    const uint32_t i = r0 + threadIdx.x;
    uint32_t res = GK_INVALID;
    if (i < n) {
        PairIdx p;
        p.r = i;
        p.pos = ld_once(a, a.cand_pos + i);
        p.e = a.e_pair ? (uint32_t)ld_once(a, a.e_pair + i) : a.e_uniform;
        PairData<W> d;
        load_window<W>(a, p.pos, d);
        const uint64_t off = read_off[i];
        // offsets that decrease give an empty read, as in the read encoder
        const uint64_t len = read_off[i + 1] >= off ? read_off[i + 1] - off : 0u;
        const uint64_t use = len < 16ull * rows ? len : 16ull * rows;     // bases encoded
        uint32_t unknown = 0;
        if (staged && off >= base && off + use <= end && use <= len) {
            const uint32_t p0 = (uint32_t)(off - a0);
            const uint32_t q = p0 >> 5, sh = p0 & 31u;
            const uint32_t u = (uint32_t)use;
            uint32_t l_prev = p_lo[q], h_prev = p_hi[q], n_prev = p_un[q];
#pragma unroll
            for (int w2 = 0; w2 < W; ++w2) {
                // 32 bases from p0 + 32 w2: plane words q + w2 and q + w2 + 1
                // (the sentinel, or text past the span, is masked below)
                const uint32_t qn = q + w2 + 1u <= nw ? q + w2 + 1u : nw;
                const uint32_t l_next = p_lo[qn], h_next = p_hi[qn], n_next = p_un[qn];
                const uint32_t have = u > 32u * w2 ? u - 32u * w2 : 0u;
                const uint32_t keep = have >= 32u ? 0xFFFFFFFFu : (1u << have) - 1u;
                const uint32_t lo = __builtin_amdgcn_alignbit(l_next, l_prev, sh) & keep;
                const uint32_t hi = __builtin_amdgcn_alignbit(h_next, h_prev, sh) & keep;
                unknown |= __builtin_amdgcn_alignbit(n_next, n_prev, sh) & keep;
                d.words[2 * w2] = (lo & 0xFFFFu) | (hi << 16);
                d.words[2 * w2 + 1] = (lo >> 16) | (hi & 0xFFFF0000u);
                l_prev = l_next;
                h_prev = h_next;
                n_prev = n_next;
            }
        } else {
#pragma unroll
            for (int j = 0; j < 2 * W; ++j)
                d.words[j] = (uint32_t)j < rows ? word_direct(ascii, off, len, 16ull * j, unknown)
                                                : 0u;
        }
        d.m = (uint32_t)(len < 0xFFFFu ? len : 0xFFFFu);
        uint32_t est;
        res = compute_pair<W, GK_READS_SPLIT, true, VAR, true>(a, p, d, est);
        // An unknown base in a read of a valid length makes the pair
        // undefined, as the read's unknown flag does for the plain launch.
        if (unknown && d.m != 0u && d.m <= a.max_read_len) {
            res = GK_UNDEFINED;
            est = GK_EST_NONE;
        }
        __builtin_nontemporal_store((uint8_t)res, a.accept + i);
        __builtin_nontemporal_store((uint16_t)est, a.est + i);
    }
    if (a.accept_bits) {
        const unsigned long long bits = __ballot(i < n && (res == GK_ACCEPT || res == GK_UNDEFINED));
        if ((threadIdx.x & 63u) == 0u && i < n)
            a.accept_bits[i >> 6] = bits;
    }
}

template <int W>
hipError_t launch_w(const FilterArgs &a, const uint8_t *ascii, const uint64_t *read_off,
                    hipStream_t s)
{
    const size_t lds = enc_lds_bytes(a.rows);
    const uint64_t CHUNK = 1ull << 30;
    for (uint64_t first = 0; first < a.n_pairs; first += CHUNK) {
        FilterArgs c = a;
        const uint64_t n = a.n_pairs - first < CHUNK ? a.n_pairs - first : CHUNK;
        c.n_pairs = n;
        c.n_reads = (uint32_t)n;
        c.cand_pos = a.cand_pos + first;
        c.e_pair = a.e_pair ? a.e_pair + first : nullptr;
        c.accept = a.accept + first;
        c.est = a.est + first;
        c.accept_bits = a.accept_bits ? a.accept_bits + first / 64 : nullptr;
        const dim3 grid((uint32_t)((n + ENC_G - 1) / ENC_G));
        if (a.flags != 0u)
            hipLaunchKernelGGL((k_filter_ascii<W, true>), grid, dim3(256), lds, s, c, ascii,
                               read_off + first);
        else
            hipLaunchKernelGGL((k_filter_ascii<W, false>), grid, dim3(256), lds, s, c, ascii,
                               read_off + first);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_filter_ascii(const FilterArgs &a, uint32_t words, const uint8_t *ascii,
                               const uint64_t *read_off, hipStream_t s)
{
    switch (words) {
    case 1: return launch_w<1>(a, ascii, read_off, s);
    case 2: return launch_w<2>(a, ascii, read_off, s);
    case 3: return launch_w<3>(a, ascii, read_off, s);
    case 4: return launch_w<4>(a, ascii, read_off, s);
    case 5: return launch_w<5>(a, ascii, read_off, s);
    case 6: return launch_w<6>(a, ascii, read_off, s);
    case 7: return launch_w<7>(a, ascii, read_off, s);
    case 8: return launch_w<8>(a, ascii, read_off, s);
    case 9: return launch_w<9>(a, ascii, read_off, s);
    case 10: return launch_w<10>(a, ascii, read_off, s);
    case 11: return launch_w<11>(a, ascii, read_off, s);
    case 12: return launch_w<12>(a, ascii, read_off, s);
    case 13: return launch_w<13>(a, ascii, read_off, s);
    case 14: return launch_w<14>(a, ascii, read_off, s);
    case 15: return launch_w<15>(a, ascii, read_off, s);
    case 16: return launch_w<16>(a, ascii, read_off, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace gkd

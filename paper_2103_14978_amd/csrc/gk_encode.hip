// Encoding kernels (Sec. 3.3 and Sec. 3.5): ASCII -> 2-bit codes A=00 C=01
// G=10 T=11 (Sec. 2.1), with every other byte recorded as an unknown base.
//   k_encode_reads     reads -> 16 bases per 32-bit word (split or interleaved
//                      code bits), transposed rows
//   k_pack_reference   reference -> two bit-planes + unknown-base plane
#include "gk_encode_dev.h"
#include "gk_internal.h"

namespace gkd {
namespace {

// One read's rows packed words straight from global memory (any alignment,
// any offsets).  Returns 1 if a byte other than A/C/G/T is among the read's
// first 16 * rows bytes.
template <uint32_t LAYOUT>
__device__ __forceinline__ uint32_t encode_direct(const uint8_t *ascii, uint64_t off, uint64_t len,
                                                  uint32_t r, uint32_t pitch, uint32_t rows,
                                                  uint32_t *packed)
{
    uint32_t unknown = 0;
    for (uint32_t w = 0; w < rows; ++w) {
        uint32_t word = 0;
        const uint64_t first = 16ull * w;
        if (first < len) {
            const uint32_t n = (uint32_t)((len - first) < 16 ? (len - first) : 16);
            uint32_t b[4];
            load16(ascii + off + first, n, b);
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const uint32_t c = (b[j >> 2] >> (8 * (j & 3))) & 0xFFu;
                if ((uint32_t)j < n) {
                    const uint32_t code = code_of(c);
                    if (LAYOUT == GK_READS_SPLIT)
                        word |= ((code & 1u) << j) | ((code >> 1) << (16 + j));
                    else
                        word |= code << (2 * j);
                    unknown |= is_base(c) ? 0u : 1u;
                }
            }
        }
        packed[(size_t)w * pitch + r] = word;
    }
    return unknown;
}

// Fallback encoder: one lane per read, straight from global memory.  Used
// when the ASCII buffer is not 16-byte aligned.  Text offset t is at
// ascii[t - text_base] (text_base <= every read_off entry).
template <uint32_t LAYOUT>
__global__ __launch_bounds__(256) void k_encode_reads(const uint8_t *ascii, uint64_t text_base,
                                                      const uint64_t *read_off, uint32_t n_reads,
                                                      uint32_t pitch, uint32_t rows,
                                                      uint32_t *packed, uint16_t *len_out,
                                                      uint8_t *has_n_out)
{
    const uint32_t r = blockIdx.x * 256u + threadIdx.x;
    if (r >= n_reads)
        return;
    const uint64_t off = read_off[r] - text_base;
    // offsets that decrease give an empty read (its pairs are GK_INVALID)
    const uint64_t len = read_off[r + 1] >= read_off[r] ? read_off[r + 1] - read_off[r] : 0u;
    const uint32_t unknown = encode_direct<LAYOUT>(ascii, off, len, r, pitch, rows, packed);
    len_out[r] = (uint16_t)(len < 0xFFFFu ? len : 0xFFFFu);
    if (has_n_out)
        has_n_out[r] = (uint8_t)unknown;
}

template <uint32_t LAYOUT>
__device__ __forceinline__ uint32_t pack_half(uint32_t lo16, uint32_t hi16)
{
    if (LAYOUT == GK_READS_SPLIT)
        return lo16 | (hi16 << 16);
    // interleaved: code bits of base j at 2j (low) and 2j+1 (high)
    uint32_t a = lo16, b = hi16;
    a = (a | (a << 8)) & 0x00FF00FFu;
    a = (a | (a << 4)) & 0x0F0F0F0Fu;
    a = (a | (a << 2)) & 0x33333333u;
    a = (a | (a << 1)) & 0x55555555u;
    b = (b | (b << 8)) & 0x00FF00FFu;
    b = (b | (b << 4)) & 0x0F0F0F0Fu;
    b = (b | (b << 2)) & 0x33333333u;
    b = (b | (b << 1)) & 0x55555555u;
    return a | (b << 1);
}

template <uint32_t LAYOUT>
__global__ __launch_bounds__(256) void k_encode_reads_staged(const uint8_t *ascii,
                                                             uint64_t text_base,
                                                             const uint64_t *read_off,
                                                             uint32_t n_reads, uint32_t pitch,
                                                             uint32_t rows, uint32_t *packed,
                                                             uint16_t *len_out,
                                                             uint8_t *has_n_out)
{
    extern __shared__ uint32_t enc_lds[];
    const uint32_t cap = enc_cap_words(rows);
    uint32_t *p_lo = enc_lds;
    uint32_t *p_hi = enc_lds + (cap + 1u);
    uint32_t *p_un = enc_lds + 2u * (cap + 1u);

    const uint32_t r0 = blockIdx.x * ENC_G;
    const uint32_t r1 = n_reads - r0 < ENC_G ? n_reads : r0 + ENC_G;
    const uint64_t base = read_off[r0] - text_base;
    const uint64_t end = read_off[r1] - text_base;
    const uint64_t a0 = base & ~31ull;                  // span start, 32-byte aligned
    // Staged when the span is in order and fits (reads longer than 16 * rows
    // bases, or offsets out of order, take the direct path).
    const bool staged = end >= base && end - a0 <= 32ull * cap;
    uint32_t nw = 0;
    if (staged) {
        nw = (uint32_t)((end - a0 + 31u) / 32u);
        for (uint32_t j = threadIdx.x; j < nw; j += 256u) {
            const uint64_t at = a0 + 32ull * j;
            const uint32_t n = end - at < 32u ? (uint32_t)(end - at) : 32u;
            uint32_t d[8];
            load_chunk(ascii + at, n, d);
            uint32_t lo, hi, un;
            chunk_planes(d, n, lo, hi, un);
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

    const uint32_t r = r0 + threadIdx.x;
    if (r >= r1)
        return;
    const uint64_t off = read_off[r] - text_base;
    // offsets that decrease give an empty read (its pairs are GK_INVALID)
    const uint64_t len = read_off[r + 1] >= read_off[r] ? read_off[r + 1] - read_off[r] : 0u;
    const uint64_t use = len < 16ull * rows ? len : 16ull * rows;     // bases encoded
    uint32_t unknown;
    if (staged && off >= base && off + use <= end && use <= len) {
        const uint32_t p0 = (uint32_t)(off - a0);
        const uint32_t q = p0 >> 5, sh = p0 & 31u;
        const uint32_t u = (uint32_t)use;
        uint32_t un_any = 0;
        uint32_t l_prev = p_lo[q], h_prev = p_hi[q], n_prev = p_un[q];
        for (uint32_t w2 = 0; 2u * w2 < rows; ++w2) {
            // 32 bases from p0 + 32 w2: words q + w2 and q + w2 + 1 (the
            // sentinel or later text past the span: masked below)
            const uint32_t qn = q + w2 + 1u <= nw ? q + w2 + 1u : nw;
            const uint32_t l_next = p_lo[qn], h_next = p_hi[qn], n_next = p_un[qn];
            uint32_t lo = __builtin_amdgcn_alignbit(l_next, l_prev, sh);
            uint32_t hi = __builtin_amdgcn_alignbit(h_next, h_prev, sh);
            uint32_t un = __builtin_amdgcn_alignbit(n_next, n_prev, sh);
            const uint32_t have = u > 32u * w2 ? u - 32u * w2 : 0u;
            const uint32_t keep = have >= 32u ? 0xFFFFFFFFu : (1u << have) - 1u;
            lo &= keep;
            hi &= keep;
            un_any |= un & keep;
            packed[(size_t)(2u * w2) * pitch + r] = pack_half<LAYOUT>(lo & 0xFFFFu, hi & 0xFFFFu);
            if (2u * w2 + 1u < rows)
                packed[(size_t)(2u * w2 + 1u) * pitch + r] = pack_half<LAYOUT>(lo >> 16, hi >> 16);
            l_prev = l_next;
            h_prev = h_next;
            n_prev = n_next;
        }
        unknown = un_any ? 1u : 0u;
    } else {
        unknown = encode_direct<LAYOUT>(ascii, off, len, r, pitch, rows, packed);
    }
    len_out[r] = (uint16_t)(len < 0xFFFFu ? len : 0xFFFFu);
    if (has_n_out)
        has_n_out[r] = (uint8_t)unknown;
}

// One thread per 32-base word.  ascii holds bases [first, first + n) and
// first is a multiple of 32, so thread t reads ascii[32t, 32t + 32).
__global__ __launch_bounds__(256) void k_pack_reference(const uint8_t *ascii, uint64_t first,
                                                        uint64_t n, uint2 *planes, uint32_t *unk,
                                                        unsigned long long *counter)
{
    const uint64_t t = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    const uint64_t nwords = (n + 31) / 32;
    uint32_t hi = 0, lo = 0, un = 0;
    if (t < nwords) {
        const uint64_t base = 32 * t;
        const uint32_t cnt = (uint32_t)((n - base) < 32 ? (n - base) : 32);
        uint32_t b0[4], b1[4];
        load16(ascii + base, cnt < 16 ? cnt : 16, b0);
        load16(ascii + base + 16, cnt > 16 ? cnt - 16 : 0, b1);
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            const uint32_t dw = j < 16 ? b0[(j >> 2) & 3] : b1[(j >> 2) & 3];
            const uint32_t c = (dw >> (8 * (j & 3))) & 0xFFu;
            if ((uint32_t)j < cnt) {
                if (is_base(c)) {
                    const uint32_t code = code_of(c);
                    hi |= (code >> 1) << j;
                    lo |= (code & 1u) << j;
                } else {
                    un |= 1u << j;
                }
            }
        }
        const uint64_t word = first / 32 + t;
        planes[word] = make_uint2(hi, lo);
        unk[word] = un;
    }
    // wave-wide sum of unknown bases, one atomic per wave
    uint32_t c = __builtin_popcount(un);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63u) == 0u && c)
        atomicAdd(counter, (unsigned long long)c);
}

// Host-encoded rows to the transposed layout.  A workgroup takes ENC_G
// reads, reads their rows * ENC_G words as one contiguous run (consecutive
// lanes, consecutive words) into LDS, and then writes each row with
// consecutive lanes.  inv_rows = ceil(2^32 / rows), so that g / rows =
// (g * inv_rows) >> 32 for every word index g of a workgroup (g < 2^13).
__global__ __launch_bounds__(256) void k_transpose_reads(const uint32_t *rowmajor,
                                                         uint32_t n_reads, uint32_t rows,
                                                         uint32_t pitch, uint64_t inv_rows,
                                                         uint32_t *out)
{
    extern __shared__ uint32_t tr_lds[];
    const uint32_t stride = rows | 1u;        // odd stride: a row's reads hit distinct banks
    const uint32_t r0 = blockIdx.x * ENC_G;
    const uint32_t nr = n_reads - r0 < ENC_G ? n_reads - r0 : ENC_G;
    const uint32_t total = nr * rows;
    const uint32_t *src = rowmajor + (size_t)r0 * rows;
    for (uint32_t g = threadIdx.x; g < total; g += 256u) {
        const uint32_t rr = (uint32_t)(((uint64_t)g * inv_rows) >> 32);
        tr_lds[rr * stride + (g - rr * rows)] = __builtin_nontemporal_load(src + g);
    }
    __syncthreads();
    const uint32_t t = threadIdx.x;
    if (t < nr)
        for (uint32_t w = 0; w < rows; ++w)
            out[(size_t)w * pitch + r0 + t] = tr_lds[t * stride + w];
}

}  // namespace

hipError_t launch_transpose_reads(const uint32_t *rowmajor, uint32_t n_reads, uint32_t rows,
                                  uint32_t pitch, uint32_t *out, hipStream_t s)
{
    if (n_reads == 0)
        return hipSuccess;
    const uint64_t inv_rows = ((1ull << 32) + rows - 1) / rows;
    hipLaunchKernelGGL(k_transpose_reads, dim3((n_reads + ENC_G - 1) / ENC_G), dim3(256),
                       (size_t)ENC_G * (rows | 1u) * 4u, s, rowmajor, n_reads, rows, pitch,
                       inv_rows, out);
    return hipGetLastError();
}

hipError_t launch_encode_reads(const uint8_t *ascii, const uint64_t *read_off, uint32_t n_reads,
                               uint32_t pitch, uint32_t rows, uint32_t layout, uint32_t *packed,
                               uint16_t *len_out, uint8_t *has_n_out, hipStream_t s,
                               uint64_t text_base)
{
    if (n_reads == 0)
        return hipSuccess;
    const bool split = layout == GK_READS_SPLIT;
    if ((((uintptr_t)ascii | text_base) & 15u) == 0u) {
        const dim3 grid((n_reads + ENC_G - 1) / ENC_G);
        const size_t lds = enc_lds_bytes(rows);
        if (split)
            hipLaunchKernelGGL(k_encode_reads_staged<GK_READS_SPLIT>, grid, dim3(256), lds, s,
                               ascii, text_base, read_off, n_reads, pitch, rows, packed, len_out,
                               has_n_out);
        else
            hipLaunchKernelGGL(k_encode_reads_staged<GK_READS_INTERLEAVED>, grid, dim3(256), lds,
                               s, ascii, text_base, read_off, n_reads, pitch, rows, packed,
                               len_out, has_n_out);
        return hipGetLastError();
    }
    const dim3 grid((n_reads + 255) / 256);
    if (split)
        hipLaunchKernelGGL(k_encode_reads<GK_READS_SPLIT>, grid, dim3(256), 0, s, ascii, text_base,
                           read_off, n_reads, pitch, rows, packed, len_out, has_n_out);
    else
        hipLaunchKernelGGL(k_encode_reads<GK_READS_INTERLEAVED>, grid, dim3(256), 0, s, ascii,
                           text_base, read_off, n_reads, pitch, rows, packed, len_out, has_n_out);
    return hipGetLastError();
}

hipError_t launch_pack_reference(const uint8_t *ascii, uint64_t first, uint64_t n, uint2 *planes,
                                 uint32_t *unk, unsigned long long *counter, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    const uint64_t nwords = (n + 31) / 32;
    hipLaunchKernelGGL(k_pack_reference, dim3((uint32_t)((nwords + 255) / 256)), dim3(256), 0, s,
                       ascii, first, n, planes, unk, counter);
    return hipGetLastError();
}

}  // namespace gkd

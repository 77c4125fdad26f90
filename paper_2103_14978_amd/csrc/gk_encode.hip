// Encoding kernels (Sec. 3.3 and Sec. 3.5): ASCII -> 2-bit codes A=00 C=01
// G=10 T=11 (Sec. 2.1), with every other byte recorded as an unknown base.
//   k_encode_reads     reads -> 16 bases per 32-bit word (split or interleaved
//                      code bits), transposed rows
//   k_pack_reference   reference -> two bit-planes + unknown-base plane
#include "gk_internal.h"

namespace gkd {
namespace {

// Code of an ASCII base: bits 1-2 of the letter give A,C,G,T -> 0,1,2,3 after
// one XOR (A=0x41, C=0x43, G=0x47, T=0x54, same in lower case).
__device__ __forceinline__ uint32_t code_of(uint32_t c) { return ((c >> 1) ^ (c >> 2)) & 3u; }

__device__ __forceinline__ bool is_base(uint32_t c)
{
    const uint32_t l = c | 0x20u;
    return l == 'a' || l == 'c' || l == 'g' || l == 't';
}

// Up to 16 bytes starting at an arbitrary address, from aligned dword loads
// that never touch a dword without a wanted byte.  Byte j of the result is
// at bits 8(j mod 4) of out[j / 4]; bytes at or beyond n are 0.
__device__ __forceinline__ void load16(const uint8_t *p, uint32_t n, uint32_t (&out)[4])
{
    const uintptr_t addr = (uintptr_t)p;
    const uint32_t *q = (const uint32_t *)(addr & ~(uintptr_t)3);
    const uint32_t sh = (uint32_t)(addr & 3u) * 8u;
    const uintptr_t end = addr + n;
    uint32_t dw[5];
#pragma unroll
    for (int j = 0; j < 5; ++j)
        dw[j] = ((uintptr_t)(q + j) < end) ? q[j] : 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        out[j] = __builtin_amdgcn_alignbit(dw[j + 1], dw[j], sh);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int lo = 4 * j;
        // clear bytes at or beyond n
        const uint32_t keep = n >= (uint32_t)(lo + 4) ? 0xFFFFFFFFu
                            : (n <= (uint32_t)lo ? 0u : ((1u << (8u * (n - lo))) - 1u));
        out[j] &= keep;
    }
}

template <uint32_t LAYOUT>
__global__ __launch_bounds__(256) void k_encode_reads(const uint8_t *ascii,
                                                      const uint64_t *read_off, uint32_t n_reads,
                                                      uint32_t pitch, uint32_t rows,
                                                      uint32_t *packed, uint16_t *len_out,
                                                      uint8_t *has_n_out)
{
    const uint32_t r = blockIdx.x * 256u + threadIdx.x;
    if (r >= n_reads)
        return;
    const uint64_t off = read_off[r];
    const uint64_t len = read_off[r + 1] - off;
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

// One lane per read: its rows consecutive words in, one word per transposed
// row out (the writes of a wave to one row are consecutive).
__global__ __launch_bounds__(256) void k_transpose_reads(const uint32_t *rowmajor,
                                                         uint32_t n_reads, uint32_t rows,
                                                         uint32_t pitch, uint32_t *out)
{
    const uint32_t r = blockIdx.x * 256u + threadIdx.x;
    if (r >= n_reads)
        return;
    const uint32_t *src = rowmajor + (size_t)r * rows;
    for (uint32_t w = 0; w < rows; ++w)
        out[(size_t)w * pitch + r] = src[w];
}

}  // namespace

hipError_t launch_transpose_reads(const uint32_t *rowmajor, uint32_t n_reads, uint32_t rows,
                                  uint32_t pitch, uint32_t *out, hipStream_t s)
{
    if (n_reads == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_transpose_reads, dim3((n_reads + 255) / 256), dim3(256), 0, s, rowmajor,
                       n_reads, rows, pitch, out);
    return hipGetLastError();
}

hipError_t launch_encode_reads(const uint8_t *ascii, const uint64_t *read_off, uint32_t n_reads,
                               uint32_t pitch, uint32_t rows, uint32_t layout, uint32_t *packed,
                               uint16_t *len_out, uint8_t *has_n_out, hipStream_t s)
{
    if (n_reads == 0)
        return hipSuccess;
    if (layout == GK_READS_SPLIT)
        hipLaunchKernelGGL(k_encode_reads<GK_READS_SPLIT>, dim3((n_reads + 255) / 256), dim3(256),
                           0, s, ascii, read_off, n_reads, pitch, rows, packed, len_out,
                           has_n_out);
    else
        hipLaunchKernelGGL(k_encode_reads<GK_READS_INTERLEAVED>, dim3((n_reads + 255) / 256),
                           dim3(256), 0, s, ascii, read_off, n_reads, pitch, rows, packed,
                           len_out, has_n_out);
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

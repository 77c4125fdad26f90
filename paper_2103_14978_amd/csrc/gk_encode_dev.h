// Device helpers of the read encoding (Sec. 3.3; codes A=00 C=01 G=10 T=11,
// Sec. 2.1) shared by the encoder kernels and the filter that encodes its own
// reads: per-byte codes, unaligned 16-byte loads, and the staging of a
// workgroup's ASCII span as three bit-planes in LDS.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace gkd {

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

// ---- staged encoder -------------------------------------------------------
//
// A workgroup takes ENC_G consecutive reads.  Their text is one contiguous
// span of the ASCII buffer; the workgroup reads it with aligned 16-byte loads
// (consecutive lanes, consecutive bytes), turns every 32 bytes into three
// 32-bit planes in LDS (low code bits, high code bits, unknown bases; base b
// of the group at bit b), and then each lane cuts its own read's words out of
// the planes with funnel shifts and writes them to the transposed rows, where
// the lanes' stores are consecutive.  The planes take a quarter of the text's
// bytes, so every read length up to 512 fits.

constexpr uint32_t ENC_G = 256;

__host__ __device__ inline uint32_t enc_cap_words(uint32_t rows)
{
    // 32-base words of the longest span staged: ENC_G reads of 16 * rows
    // bases, plus one word for the span's start alignment.
    return ENC_G * 16u * rows / 32u + 1u;
}

// Bytes of dynamic LDS: three planes of cap + 1 words (the extra word is a
// zero sentinel after the span).
__host__ inline size_t enc_lds_bytes(uint32_t rows) { return 3u * (enc_cap_words(rows) + 1u) * 4u; }

// The 32 bytes of a staging chunk at p (16-byte aligned).  Bytes at or beyond
// `n` are not needed; dwords holding none of the first n bytes are not read.
__device__ __forceinline__ void load_chunk(const uint8_t *p, uint32_t n, uint32_t (&d)[8])
{
    if (n >= 32u) {
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        const u32x4 a = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
        const u32x4 b = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p) + 1);
        d[0] = a.x, d[1] = a.y, d[2] = a.z, d[3] = a.w;
        d[4] = b.x, d[5] = b.y, d[6] = b.z, d[7] = b.w;
    } else {
        const uint32_t *q = reinterpret_cast<const uint32_t *>(p);
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j)
            d[j] = 4u * j < n ? q[j] : 0u;
    }
}

// Planes of 32 ASCII bytes (d[i] holds bytes 4i .. 4i+3, byte 4i+k at bits
// 8k).  A base's code is bits 1-2 of (c ^ (c >> 1)) for the letters
// A C G T a c g t; a byte is a base iff it equals, up to case, the letter its
// code names.  Bits of the four bytes of a dword are gathered with a byte dot
// product against powers of two.
__device__ __forceinline__ void chunk_planes(const uint32_t (&d)[8], uint32_t n, uint32_t &lo,
                                             uint32_t &hi, uint32_t &un)
{
    uint32_t x[8], bad_any = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        x[i] = d[i] ^ (d[i] >> 1);
        // the letter (lower case) each byte's code names: codes 0..3 select
        // bytes 0 and 2 of the second operand, 0 and 2 of the first
        const uint32_t letter = __builtin_amdgcn_perm(0x00740067u, 0x00630061u, x[i] & 0x06060606u);
        bad_any |= (d[i] ^ letter) & 0xDFDFDFDFu;
    }
    // byte j of the result: the pair of dwords 2j, 2j+1 (bits of value 2 or 4)
    uint32_t bl[4], bh[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        bl[j] = __builtin_amdgcn_udot4(x[2 * j] & 0x02020202u, 0x08040201u,
                                       __builtin_amdgcn_udot4(x[2 * j + 1] & 0x02020202u,
                                                              0x80402010u, 0u, false),
                                       false);
        bh[j] = __builtin_amdgcn_udot4(x[2 * j] & 0x04040404u, 0x08040201u,
                                       __builtin_amdgcn_udot4(x[2 * j + 1] & 0x04040404u,
                                                              0x80402010u, 0u, false),
                                       false);
    }
    // bl[j] = 2 * byte, bh[j] = 4 * byte
    lo = (bl[0] >> 1) | (bl[1] << 7) | (bl[2] << 15) | (bl[3] << 23);
    hi = (bh[0] >> 2) | (bh[1] << 6) | (bh[2] << 14) | (bh[3] << 22);
    un = 0;
    if (bad_any) {
        // per byte: 1 if it differs from its letter in any bit but the case bit
        uint32_t bu[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            uint32_t f[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int i = 2 * j + h;
                const uint32_t letter =
                    __builtin_amdgcn_perm(0x00740067u, 0x00630061u, x[i] & 0x06060606u);
                const uint32_t mm = (d[i] ^ letter) & 0xDFDFDFDFu;
                f[h] = ((((mm & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | mm) >> 7) & 0x01010101u;
            }
            bu[j] = __builtin_amdgcn_udot4(f[0], 0x08040201u,
                                           __builtin_amdgcn_udot4(f[1], 0x80402010u, 0u, false),
                                           false);
        }
        un = bu[0] | (bu[1] << 8) | (bu[2] << 16) | (bu[3] << 24);
    }
    if (n < 32u) {
        const uint32_t keep = (1u << n) - 1u;
        lo &= keep;
        hi &= keep;
        un &= keep;
    }
}

}  // namespace gkd

// Host-side read encoding for gk_filter_host (the paper's "encoding in the
// host" option, Sec. 3.3): ASCII reads -> 2-bit codes A=00 C=01 G=10 T=11
// (Sec. 2.1), 16 bases per 32-bit word with the low code bits in bits 0-15
// and the high code bits in bits 16-31, one row of words per read, plus the
// read's length and whether it holds an unknown base.  The words equal those
// k_encode_reads writes on the GPU, so either encoder gives the same filter
// results.  Host code only (x86-64): SSE2, plus an AVX2 path taken when the
// CPU has it (32 bytes, two words, per step).
#include <immintrin.h>

#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "gk_host_encode.h"

namespace {

// Low code bits, high code bits and non-base bytes of 16 ASCII bytes, as
// 16-bit masks (bit j = byte j).  The code of a letter is bits 1-2 of its
// byte XORed (A=0x41, C=0x43, G=0x47, T=0x54, same in lower case), so the low
// code bit is bit 1 ^ bit 2 and the high code bit is bit 2 ^ bit 3; the shifts
// bring those bits to bit 7 of each byte for movemask (16-bit shifts only
// disturb bits other than 7 and 15 across the byte boundary).
inline void masks16(__m128i v, uint32_t &lo, uint32_t &hi, uint32_t &other)
{
    const __m128i s4 = _mm_slli_epi16(v, 4), s5 = _mm_slli_epi16(v, 5),
                  s6 = _mm_slli_epi16(v, 6);
    lo = (uint32_t)_mm_movemask_epi8(_mm_xor_si128(s6, s5));
    hi = (uint32_t)_mm_movemask_epi8(_mm_xor_si128(s5, s4));
    const __m128i l = _mm_or_si128(v, _mm_set1_epi8(0x20));
    const __m128i base =
        _mm_or_si128(_mm_or_si128(_mm_cmpeq_epi8(l, _mm_set1_epi8('a')),
                                  _mm_cmpeq_epi8(l, _mm_set1_epi8('c'))),
                     _mm_or_si128(_mm_cmpeq_epi8(l, _mm_set1_epi8('g')),
                                  _mm_cmpeq_epi8(l, _mm_set1_epi8('t'))));
    other = ~(uint32_t)_mm_movemask_epi8(base) & 0xFFFFu;
}

// The same three masks for 32 bytes (bit j = byte j).
__attribute__((target("avx2"))) inline void masks32(__m256i v, uint32_t &lo, uint32_t &hi,
                                                     uint32_t &other)
{
    const __m256i s4 = _mm256_slli_epi16(v, 4), s5 = _mm256_slli_epi16(v, 5),
                  s6 = _mm256_slli_epi16(v, 6);
    lo = (uint32_t)_mm256_movemask_epi8(_mm256_xor_si256(s6, s5));
    hi = (uint32_t)_mm256_movemask_epi8(_mm256_xor_si256(s5, s4));
    const __m256i l = _mm256_or_si256(v, _mm256_set1_epi8(0x20));
    const __m256i base =
        _mm256_or_si256(_mm256_or_si256(_mm256_cmpeq_epi8(l, _mm256_set1_epi8('a')),
                                        _mm256_cmpeq_epi8(l, _mm256_set1_epi8('c'))),
                        _mm256_or_si256(_mm256_cmpeq_epi8(l, _mm256_set1_epi8('g')),
                                        _mm256_cmpeq_epi8(l, _mm256_set1_epi8('t'))));
    other = ~(uint32_t)_mm256_movemask_epi8(base);
}

// Word w of a read from its bytes [16w, 16w + n), n = 1..16.
inline uint32_t encode_word16(const uint8_t *ascii, uint64_t text_bytes, uint64_t at, uint32_t n,
                              uint32_t &unknown)
{
    const uint8_t *p = ascii + at;
    __m128i v;
    if (at + 16 <= text_bytes) {
        v = _mm_loadu_si128(reinterpret_cast<const __m128i *>(p));
    } else {                                   // never read past the caller's text
        alignas(16) uint8_t tmp[16] = {};
        std::memcpy(tmp, p, n);
        v = _mm_load_si128(reinterpret_cast<const __m128i *>(tmp));
    }
    uint32_t lo, hi, other;
    masks16(v, lo, hi, other);
    const uint32_t valid = n == 16 ? 0xFFFFu : ((1u << n) - 1u);
    unknown |= other & valid;
    return (lo & valid) | ((hi & valid) << 16);
}

void encode_rows_sse2(const uint8_t *ascii, uint64_t text_bytes, const uint64_t *read_off,
                      uint64_t r0, uint64_t r1, uint32_t rows, uint32_t *rows_out,
                      uint16_t *len_out, uint8_t *has_n_out)
{
    for (uint64_t r = r0; r < r1; ++r) {
        const uint64_t off = read_off[r];
        const uint64_t len = read_off[r + 1] - off;
        uint32_t *row = rows_out + (r - r0) * rows;
        uint32_t unknown = 0;
        for (uint32_t w = 0; w < rows; ++w) {
            const uint64_t first = 16ull * w;
            row[w] = first < len ? encode_word16(ascii, text_bytes, off + first,
                                                 (uint32_t)(len - first < 16 ? len - first : 16),
                                                 unknown)
                                 : 0u;
        }
        len_out[r - r0] = (uint16_t)(len < 0xFFFFu ? len : 0xFFFFu);
        has_n_out[r - r0] = unknown ? 1u : 0u;
    }
}

__attribute__((target("avx2"))) void encode_rows_avx2(const uint8_t *ascii, uint64_t text_bytes,
                                                      const uint64_t *read_off, uint64_t r0,
                                                      uint64_t r1, uint32_t rows,
                                                      uint32_t *rows_out, uint16_t *len_out,
                                                      uint8_t *has_n_out)
{
    for (uint64_t r = r0; r < r1; ++r) {
        const uint64_t off = read_off[r];
        const uint64_t len = read_off[r + 1] - off;
        uint32_t *row = rows_out + (r - r0) * rows;
        uint32_t unknown = 0;
        uint32_t w = 0;
        // two full words from one 32-byte load while both lie in the read
        for (; w + 1 < rows && 16ull * w + 32 <= len && off + 16ull * w + 32 <= text_bytes;
             w += 2) {
            const __m256i v =
                _mm256_loadu_si256(reinterpret_cast<const __m256i *>(ascii + off + 16ull * w));
            uint32_t lo, hi, other;
            masks32(v, lo, hi, other);
            row[w] = (lo & 0xFFFFu) | (hi << 16);
            row[w + 1] = (lo >> 16) | (hi & 0xFFFF0000u);
            unknown |= other;
        }
        for (; w < rows; ++w) {
            const uint64_t first = 16ull * w;
            row[w] = first < len ? encode_word16(ascii, text_bytes, off + first,
                                                 (uint32_t)(len - first < 16 ? len - first : 16),
                                                 unknown)
                                 : 0u;
        }
        len_out[r - r0] = (uint16_t)(len < 0xFFFFu ? len : 0xFFFFu);
        has_n_out[r - r0] = unknown ? 1u : 0u;
    }
}

}  // namespace

namespace gkd {

void host_encode_rows(const uint8_t *ascii, uint64_t text_bytes, const uint64_t *read_off,
                      uint64_t r0, uint64_t r1, uint32_t rows, uint32_t *rows_out,
                      uint16_t *len_out, uint8_t *has_n_out)
{
    static const bool avx2 = __builtin_cpu_supports("avx2");
    if (avx2)
        encode_rows_avx2(ascii, text_bytes, read_off, r0, r1, rows, rows_out, len_out,
                         has_n_out);
    else
        encode_rows_sse2(ascii, text_bytes, read_off, r0, r1, rows, rows_out, len_out,
                         has_n_out);
}

void host_encode_rows_sse2(const uint8_t *ascii, uint64_t text_bytes, const uint64_t *read_off,
                           uint64_t r0, uint64_t r1, uint32_t rows, uint32_t *rows_out,
                           uint16_t *len_out, uint8_t *has_n_out)
{
    encode_rows_sse2(ascii, text_bytes, read_off, r0, r1, rows, rows_out, len_out, has_n_out);
}

struct HostEncodePool::State {
    std::vector<std::thread> threads;
    std::mutex mu;
    std::condition_variable go, done;
    std::function<void(unsigned, unsigned)> task;
    uint64_t generation = 0;
    unsigned pending = 0;
    bool quit = false;
};

HostEncodePool::HostEncodePool(unsigned n) : s_(new State)
{
    State *s = s_;
    for (unsigned i = 0; i < n; ++i)
        s->threads.emplace_back([s, i, n] {
            uint64_t seen = 0;
            for (;;) {
                std::function<void(unsigned, unsigned)> fn;
                {
                    std::unique_lock<std::mutex> lk(s->mu);
                    s->go.wait(lk, [&] { return s->quit || s->generation != seen; });
                    if (s->quit)
                        return;
                    seen = s->generation;
                    fn = s->task;
                }
                fn(i, n);
                std::lock_guard<std::mutex> lk(s->mu);
                if (--s->pending == 0)
                    s->done.notify_one();
            }
        });
}

HostEncodePool::~HostEncodePool()
{
    {
        std::lock_guard<std::mutex> lk(s_->mu);
        s_->quit = true;
    }
    s_->go.notify_all();
    for (std::thread &t : s_->threads)
        t.join();
    delete s_;
}

void HostEncodePool::run(const std::function<void(unsigned, unsigned)> &fn)
{
    std::unique_lock<std::mutex> lk(s_->mu);
    s_->task = fn;
    s_->pending = (unsigned)s_->threads.size();
    ++s_->generation;
    s_->go.notify_all();
    s_->done.wait(lk, [&] { return s_->pending == 0; });
}

}  // namespace gkd

extern "C" void gk_detail_host_encode_rows(const uint8_t *ascii, const uint64_t *read_off,
                                           uint64_t n_reads, uint32_t rows, uint32_t *rows_out,
                                           uint16_t *len_out, uint8_t *has_n_out, int sse2_only)
{
    if (n_reads == 0)
        return;
    (sse2_only ? gkd::host_encode_rows_sse2 : gkd::host_encode_rows)(
        ascii, read_off[n_reads], read_off, 0, n_reads, rows, rows_out, len_out, has_n_out);
}

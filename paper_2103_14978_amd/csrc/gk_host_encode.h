// Host-side read encoding for gk_filter_host (host code only).
#pragma once

#include <cstdint>
#include <functional>

namespace gkd {

// Encodes reads [r0, r1) of an ASCII batch: read r's bases are
// ascii[read_off[r], read_off[r + 1]), text_bytes = read_off[n_reads] bounds
// every load.  Row r - r0 of rows_out gets `rows` words of 16 bases each
// (low code bits in bits 0-15, high in bits 16-31; bases past the read are 0),
// len_out the read length (capped at 65535) and has_n_out 1 if a byte among
// the first 16 * rows is not A/C/G/T (either case) — the same as the GPU
// encoder writes.
void host_encode_rows(const uint8_t *ascii, uint64_t text_bytes, const uint64_t *read_off,
                      uint64_t r0, uint64_t r1, uint32_t rows, uint32_t *rows_out,
                      uint16_t *len_out, uint8_t *has_n_out);
// The same with the SSE2 path only (host_encode_rows takes AVX2 when the CPU
// has it).
void host_encode_rows_sse2(const uint8_t *ascii, uint64_t text_bytes, const uint64_t *read_off,
                           uint64_t r0, uint64_t r1, uint32_t rows, uint32_t *rows_out,
                           uint16_t *len_out, uint8_t *has_n_out);

// A fixed set of worker threads: run(fn) calls fn(i, n) on each of the n
// workers and returns when all have returned.  One caller thread at a time.
class HostEncodePool {
  public:
    explicit HostEncodePool(unsigned n);
    ~HostEncodePool();
    HostEncodePool(const HostEncodePool &) = delete;
    HostEncodePool &operator=(const HostEncodePool &) = delete;
    void run(const std::function<void(unsigned, unsigned)> &fn);

  private:
    struct State;
    State *s_;
};

}  // namespace gkd

// For tests of the host logic (no GPU needed): gkd::host_encode_rows (or,
// with sse2_only, gkd::host_encode_rows_sse2) on reads [0, n_reads).
extern "C" void gk_detail_host_encode_rows(const uint8_t *ascii, const uint64_t *read_off,
                                           uint64_t n_reads, uint32_t rows, uint32_t *rows_out,
                                           uint16_t *len_out, uint8_t *has_n_out, int sse2_only);

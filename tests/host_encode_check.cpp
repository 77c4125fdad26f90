// Sanitizer driver for the host-side read encoder and its worker pool (host
// code only).  tests/test_host_sanitizers.py builds it with the address /
// undefined-behaviour and thread sanitizers and runs it on the CPU.
//   - Text buffers are allocated at exactly read_off[n] bytes, so any load
//     past the caller's text is reported.
//   - The default path (AVX2 where the CPU has it) must equal the SSE2 path.
//   - The pool encodes the same batch in parallel parts, several times in a
//     row, and must give the same rows.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "gk_host_encode.h"

int main()
{
    std::mt19937_64 rng(20240611u);
    static const char alphabet[] = "ACGTACGTACGTacgtNn-.";
    for (int round = 0; round < 40; ++round) {
        const uint32_t rows = 1u + (uint32_t)(rng() % 32u);
        const uint64_t n = 1u + rng() % 3000u;
        std::vector<uint64_t> off(n + 1, 0);
        for (uint64_t i = 0; i < n; ++i)
            off[i + 1] = off[i] + rng() % (16u * rows + 40u);
        const uint64_t bytes = off[n];
        uint8_t *text = static_cast<uint8_t *>(std::malloc(bytes ? bytes : 1));
        for (uint64_t i = 0; i < bytes; ++i)
            text[i] = (uint8_t)alphabet[rng() % (sizeof(alphabet) - 1)];

        std::vector<uint32_t> a(n * rows), b(n * rows), c(n * rows);
        std::vector<uint16_t> la(n), lb(n), lc(n);
        std::vector<uint8_t> ha(n), hb(n), hc(n);
        gkd::host_encode_rows(text, bytes, off.data(), 0, n, rows, a.data(), la.data(),
                              ha.data());
        gkd::host_encode_rows_sse2(text, bytes, off.data(), 0, n, rows, b.data(), lb.data(),
                                   hb.data());
        if (a != b || la != lb || ha != hb) {
            std::printf("round %d: default and SSE2 paths differ\n", round);
            return 1;
        }
        gkd::HostEncodePool pool(1u + (unsigned)(round % 8));
        for (int rep = 0; rep < 5; ++rep) {
            std::fill(c.begin(), c.end(), 0xDEADBEEFu);
            pool.run([&](unsigned i, unsigned k) {
                const uint64_t s = n * i / k, e = n * (i + 1) / k;
                gkd::host_encode_rows(text, bytes, off.data(), s, e, rows, c.data() + s * rows,
                                      lc.data() + s, hc.data() + s);
            });
            if (c != a || lc != la || hc != ha) {
                std::printf("round %d rep %d: pool result differs\n", round, rep);
                return 1;
            }
        }
        std::free(text);
    }
    std::puts("host encode check ok");
    return 0;
}

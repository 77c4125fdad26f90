// CPU driver for the host-to-host pipeline's host logic (gk_host.hip built as
// host C++), against the stand-in HIP runtime of standin_hip.h with random
// delays before every stream operation: no GPU.  tests/test_host_pipe.py
// builds it plain and under the address / undefined-behaviour and thread
// sanitizers.
//
// The stand-in read encoder writes the words the library's host encoder
// writes (gkd::host_encode_rows), transposed; the stand-in filter writes, for
// every pair, a fixed function of its read's words, length and unknown flag,
// its position and its threshold.  A pair filtered against the wrong read,
// chunk or slot, or results taken from a slot before its filter ended or
// after the next chunk reused it, shows up as a mismatch.
//
// Checks: one pair per read (reads travel in the ring's slots), pairs in read
// order and shuffled (every read resident), pair indices past the reads,
// ASCII reads encoded on the device or on host threads, host-encoded rows
// with and without unknown flags, per-pair and uniform thresholds, chunks of
// 64 pairs up to the whole batch; the peak device memory of one-pair-per-read
// batches stays within three chunks; bad offsets are GK_EINVAL and leave the
// context usable.
#include "standin_hip.h"

#include <cstdio>
#include <numeric>

// ---- stand-in kernels -------------------------------------------------------

namespace {

uint32_t mix(uint32_t h, uint32_t v) { return (h ^ v) * 16777619u; }

// The stand-in filter result of one pair.
void expected(uint32_t words_hash, uint32_t len, uint32_t has_n, uint32_t pos, uint32_t e,
              uint8_t *acc, uint16_t *est)
{
    const uint32_t h = mix(mix(mix(mix(words_hash, len), has_n), pos), e);
    *acc = (uint8_t)(h % 3u);
    *est = (uint16_t)(h >> 16);
}

std::atomic<int> g_bad_batch{0};      // gk_filter called with inconsistent arguments

}  // namespace

extern "C" int gk_filter(gk_ctx *, const gk_batch *b, void *stream)
{
    const uint32_t rows = (b->max_read_len + 15) / 16;
    if (b->pitch < b->n_reads || (b->n_reads && (!b->reads || !b->read_len)) ||
        !b->cand_pos || !b->accept || !b->est || b->accept_bits)
        g_bad_batch++;
    const gk_batch c = *b;
    static_cast<hipStream_t>(stream)->enqueue([c, rows] {
        for (uint64_t i = 0; i < c.n_pairs; ++i) {
            const uint32_t r = c.pair_read ? c.pair_read[i] : (uint32_t)i;
            if (r >= c.n_reads) {
                c.accept[i] = GK_INVALID;
                c.est[i] = GK_EST_NONE;
                continue;
            }
            uint32_t h = 2166136261u;
            for (uint32_t w = 0; w < rows; ++w)
                h = mix(h, c.reads[(size_t)w * c.pitch + r]);
            expected(h, c.read_len[r], c.read_has_n ? c.read_has_n[r] : 0u, c.cand_pos[i],
                     c.e ? c.e[i] : c.e_uniform, &c.accept[i], &c.est[i]);
        }
    });
    return GK_OK;
}

namespace gkd {

hipError_t launch_encode_reads(const uint8_t *ascii, const uint64_t *read_off, uint32_t n_reads,
                               uint32_t pitch, uint32_t rows, uint32_t, uint32_t *packed,
                               uint16_t *len_out, uint8_t *has_n_out, hipStream_t s,
                               uint64_t text_base)
{
    s->enqueue([=] {
        std::vector<uint64_t> off(n_reads + 1);
        for (uint32_t r = 0; r <= n_reads; ++r)
            off[r] = read_off[r] - text_base;
        std::vector<uint32_t> words((size_t)n_reads * rows);
        std::vector<uint8_t> has_n(n_reads);
        host_encode_rows(ascii, off[n_reads], off.data(), 0, n_reads, rows, words.data(), len_out,
                         has_n.data());
        for (uint32_t r = 0; r < n_reads; ++r) {
            for (uint32_t w = 0; w < rows; ++w)
                packed[(size_t)w * pitch + r] = words[(size_t)r * rows + w];
            if (has_n_out)
                has_n_out[r] = has_n[r];
        }
    });
    return hipSuccess;
}

hipError_t launch_transpose_reads(const uint32_t *rowmajor, uint32_t n_reads, uint32_t rows,
                                  uint32_t pitch, uint32_t *out, hipStream_t s)
{
    s->enqueue([=] {
        for (uint32_t r = 0; r < n_reads; ++r)
            for (uint32_t w = 0; w < rows; ++w)
                out[(size_t)w * pitch + r] = rowmajor[(size_t)r * rows + w];
    });
    return hipSuccess;
}

}  // namespace gkd

// ---- checks -----------------------------------------------------------------

namespace {

int g_failures = 0;

#define CHECK(cond, ...)                                   \
    do {                                                   \
        if (!(cond)) {                                     \
            std::printf("FAIL %s:%d: ", __FILE__, __LINE__); \
            std::printf(__VA_ARGS__);                      \
            std::printf("\n");                             \
            g_failures++;                                  \
        }                                                  \
    } while (0)

struct Batch {
    uint32_t max_len = 0, rows = 0;
    std::vector<uint8_t> ascii;
    std::vector<uint64_t> off;
    std::vector<uint32_t> words;       // row-major, rows per read
    std::vector<uint16_t> len;
    std::vector<uint8_t> has_n;
    std::vector<uint32_t> pair_read, pos;
    std::vector<uint8_t> e;
};

Batch make_batch(std::mt19937_64 &rng, uint32_t n_reads, uint32_t max_len)
{
    Batch b;
    b.max_len = max_len;
    b.rows = (max_len + 15) / 16;
    b.off.push_back(0);
    const char bases[] = "ACGTacgtN";
    for (uint32_t r = 0; r < n_reads; ++r) {
        const uint32_t m = (uint32_t)(rng() % (max_len + 1));      // 0..max_len
        for (uint32_t i = 0; i < m; ++i) {
            const uint32_t k = (uint32_t)(rng() % 1000);
            b.ascii.push_back((uint8_t)bases[k < 2 ? 8 : (k < 60 ? 4 + k % 4 : k % 4)]);
        }
        b.off.push_back(b.ascii.size());
    }
    b.words.resize((size_t)n_reads * b.rows);
    b.len.resize(n_reads);
    b.has_n.resize(n_reads);
    gkd::host_encode_rows(b.ascii.data(), b.ascii.size(), b.off.data(), 0, n_reads, b.rows,
                          b.words.data(), b.len.data(), b.has_n.data());
    return b;
}

enum class Order { Identity, Sorted, Shuffled };

void make_pairs(std::mt19937_64 &rng, Batch &b, Order order, uint64_t n_pairs, bool per_pair_e)
{
    const uint32_t nr = (uint32_t)b.len.size();
    b.pair_read.clear();
    if (order == Order::Identity) {
        n_pairs = nr;
    } else {
        for (uint64_t i = 0; i < n_pairs; ++i)    // a few indices past the reads
            b.pair_read.push_back((uint32_t)(rng() % (nr + nr / 50 + 1)));
        if (order == Order::Sorted)
            std::sort(b.pair_read.begin(), b.pair_read.end());
    }
    b.pos.resize(n_pairs);
    for (auto &p : b.pos)
        p = (uint32_t)rng();
    b.e.clear();
    if (per_pair_e) {
        b.e.resize(n_pairs);
        for (auto &v : b.e)
            v = (uint8_t)(rng() % 32);
    }
}

struct Mode {
    bool host_encoded = false;     // caller-encoded rows instead of ASCII
    bool with_has_n = true;        // host-encoded rows come with unknown flags
    uint32_t threads = 0;          // GK_OPT_HOST_ENCODE_THREADS
    uint64_t chunk = 0;            // GK_OPT_HOST_CHUNK_PAIRS
};

// Runs gk_filter_host on b and compares every pair with the stand-in
// filter's function of the caller's reads.  Returns the status.
int run(gk_ctx *ctx, const Batch &b, const Mode &md, const char *label, bool compare = true)
{
    const uint64_t np = b.pos.size();
    const bool identity = b.pair_read.empty();
    ctx->host_encode_threads = md.threads;
    ctx->host_chunk_pairs = md.chunk;
    std::vector<uint8_t> acc(np, 0xEE);
    std::vector<uint16_t> est(np, 0xEEEE);
    gk_host_batch hb{};
    hb.n_reads = (uint32_t)b.len.size();
    hb.max_read_len = b.max_len;
    hb.n_pairs = np;
    hb.pair_read = identity ? nullptr : b.pair_read.data();
    hb.cand_pos = b.pos.data();
    hb.e = b.e.empty() ? nullptr : b.e.data();
    hb.e_uniform = 7;
    hb.accept = acc.data();
    hb.est = est.data();
    if (md.host_encoded) {
        hb.packed = b.words.data();
        hb.read_len = b.len.data();
        hb.read_has_n = md.with_has_n ? b.has_n.data() : nullptr;
        hb.packed_layout = GK_READS_SPLIT;
    } else {
        hb.ascii = b.ascii.data();
        hb.read_off = b.off.data();
    }
    const int st = gk_filter_host(ctx, &hb);
    if (st != GK_OK || !compare)
        return st;
    uint64_t bad = 0, first = np;
    for (uint64_t i = 0; i < np; ++i) {
        const uint32_t r = identity ? (uint32_t)i : b.pair_read[i];
        uint8_t wa = GK_INVALID;
        uint16_t we = GK_EST_NONE;
        if (r < b.len.size()) {
            uint32_t h = 2166136261u;
            for (uint32_t w = 0; w < b.rows; ++w)
                h = mix(h, b.words[(size_t)r * b.rows + w]);
            const uint32_t hn = (md.host_encoded && !md.with_has_n) ? 0u : b.has_n[r];
            expected(h, b.len[r], hn, b.pos[i], b.e.empty() ? 7u : b.e[i], &wa, &we);
        }
        if (acc[i] != wa || est[i] != we) {
            if (!bad)
                first = i;
            bad++;
        }
    }
    CHECK(bad == 0, "%s: %llu of %llu pairs differ, first %llu", label, (unsigned long long)bad,
          (unsigned long long)np, (unsigned long long)first);
    return st;
}

}  // namespace

int main()
{
    g_jitter_us = 40;
    std::mt19937_64 rng(20240611);
    uint2 ref_word{};
    gk_ctx ctx;
    ctx.ref_planes = &ref_word;       // only its presence is checked here
    ctx.ref_len = 1;

    // Per variant: chunk pairs (0 = automatic), read length bound.
    const uint64_t chunks[5] = {64, 256, 1000, 0, 128};
    const uint32_t max_lens[5] = {100, 150, 33, 250, 16};
    int cases = 0;
    for (Order order : {Order::Identity, Order::Sorted, Order::Shuffled}) {
        for (int variant = 0; variant < 5; ++variant) {
            Mode md;
            md.chunk = chunks[variant];
            md.threads = variant == 1 || variant == 4 ? 3 : 0;
            md.host_encoded = variant == 2 || variant == 3;
            md.with_has_n = variant != 3;
            const uint32_t max_len = max_lens[variant];
            Batch b = make_batch(rng, 1500 + (uint32_t)(rng() % 3000), max_len);
            make_pairs(rng, b, order, 4000 + rng() % 5000, variant % 2 == 0);
            char label[160];
            std::snprintf(label, sizeof label,
                          "order %d chunk %llu threads %u host-encoded %d has_n %d len %u", (int)order,
                          (unsigned long long)md.chunk, md.threads, (int)md.host_encoded,
                          (int)md.with_has_n, max_len);
            gk_detail_free_host_pipe(&ctx);
            {
                std::lock_guard<std::mutex> lk(g_alloc_mu);
                g_alloc_peak = g_alloc_bytes;
            }
            const int st = run(&ctx, b, md, label);
            CHECK(st == GK_OK, "%s: status %d (%s)", label, st, ctx.err.c_str());
            cases++;
            if (order == Order::Identity && md.chunk) {
                // Three slots of at most one chunk of pairs and reads each.
                const uint64_t P = (md.chunk + 63) / 64 * 64;
                const uint64_t bound = 3 * (P * (8 + 8 + 2 + 1 + 4ull * b.rows + b.max_len) +
                                            8 + 128);
                size_t peak;
                {
                    std::lock_guard<std::mutex> lk(g_alloc_mu);
                    peak = g_alloc_peak;
                }
                CHECK(peak <= bound, "%s: peak device bytes %zu above three chunks (%llu)", label,
                      peak, (unsigned long long)bound);
            }
        }
    }

    // A batch smaller than one chunk, and pairs with no reads at all.
    {
        Batch b = make_batch(rng, 5, 64);
        make_pairs(rng, b, Order::Identity, 0, false);
        ctx.log = 1;            // one log line through the stand-in's logger
        run(&ctx, b, Mode{}, "five reads, one pair each");
        ctx.log = 0;
        Batch z = make_batch(rng, 0, 64);
        make_pairs(rng, z, Order::Sorted, 300, true);
        Mode md;
        md.chunk = 64;
        run(&ctx, z, md, "no reads");
        cases += 2;
    }

    // Offsets that decrease in a late chunk: GK_EINVAL, then the context works.
    for (uint32_t threads : {0u, 2u}) {
        Batch b = make_batch(rng, 3000, 100);
        make_pairs(rng, b, Order::Identity, 0, false);
        Batch bad = b;
        CHECK(bad.off[2499] > 0, "reads before 2499 are empty");
        bad.off[2500] = bad.off[2499] - 1;
        Mode md;
        md.chunk = 256;
        md.threads = threads;
        const int st = run(&ctx, bad, md, "decreasing offsets", false);
        CHECK(st == GK_EINVAL, "decreasing offsets (threads %u): status %d", threads, st);
        run(&ctx, b, md, "after decreasing offsets");
        cases += 2;
    }

    gk_detail_free_host_pipe(&ctx);
    CHECK(g_bad_batch.load() == 0, "%d filter calls with inconsistent arguments",
          g_bad_batch.load());
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        CHECK(g_alloc_bytes == 0, "%zu device bytes still allocated", g_alloc_bytes);
    }
    if (g_failures) {
        std::printf("host pipe check: %d failures\n", g_failures);
        return 1;
    }
    std::printf("host pipe check ok: %d cases\n", cases);
    return 0;
}

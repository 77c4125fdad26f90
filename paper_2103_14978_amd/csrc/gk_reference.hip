// Resident reference from 2-bit words the caller already holds (Sec. 3.3:
// 16 bases per 32-bit word) plus a list of unknown-base runs (Sec. 3.5
// records where the reference has unknown bases).  The result is the same
// bit-plane reference and unknown-base plane that k_pack_reference builds
// from ASCII text.
#include "gk_pair.h"
#include "gk_reference.h"

namespace gkd {
namespace {

// One thread per 32-base word: two packed words -> the high and low planes.
template <int L>
__global__ __launch_bounds__(256) void k_unpack_reference(const uint32_t *packed, uint64_t first,
                                                          uint64_t n, uint2 *planes)
{
    const uint64_t t = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    const uint64_t nwords = (n + 31) / 32;
    if (t >= nwords)
        return;
    const uint64_t base = 32 * t;
    const uint64_t cnt = n - base < 32 ? n - base : 32;
    const uint32_t p0 = packed[2 * t];
    const uint32_t p1 = cnt > 16 ? packed[2 * t + 1] : 0u;
    uint32_t hi, lo;
    planes_from_words<L>(p0, p1, hi, lo);
    const uint32_t keep = ones_below((int)cnt);
    planes[first / 32 + t] = make_uint2(hi & keep, lo & keep);
}

// Blocks walk the runs; the threads of a block share one run's words.  Word
// updates are atomic ORs, so overlapping runs and runs sharing an edge word
// compose.
__global__ __launch_bounds__(256) void k_mark_runs(const uint64_t *runs, uint64_t n_runs,
                                                   uint32_t *unk)
{
    for (uint64_t r = blockIdx.x; r < n_runs; r += gridDim.x) {
        const uint64_t s = runs[2 * r], len = runs[2 * r + 1];
        if (len == 0)
            continue;
        const uint64_t e = s + len;
        const uint64_t w0 = s / 32, w1 = (e - 1) / 32;
        for (uint64_t w = w0 + threadIdx.x; w <= w1; w += 256) {
            const uint64_t lo = (s > 32 * w ? s : 32 * w) - 32 * w;
            const uint64_t hi = (e < 32 * w + 32 ? e : 32 * w + 32) - 32 * w;
            const uint32_t mask = ones_below((int)hi) & ~ones_below((int)lo);
            atomicOr(unk + w, mask);
        }
    }
}

__global__ __launch_bounds__(256) void k_count_unknown(const uint32_t *unk, uint64_t words,
                                                       unsigned long long *counter)
{
    uint32_t c = 0;
    for (uint64_t w = (uint64_t)blockIdx.x * 256u + threadIdx.x; w < words;
         w += (uint64_t)gridDim.x * 256u)
        c += __builtin_popcount(unk[w]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63u) == 0u && c)
        atomicAdd(counter, (unsigned long long)c);
}

// One lane per 512-base line of the reference; a wave's 64 answers make one
// 64-bit word of the summary.
__global__ __launch_bounds__(256) void k_unknown_lines(const uint32_t *unk, uint64_t words,
                                                       unsigned long long *lines)
{
    const uint64_t line = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    const uint64_t nlines = (words + LINE_WORDS - 1) / LINE_WORDS;
    uint32_t any = 0;
    if (line < nlines) {
        const uint64_t w0 = line * LINE_WORDS;
        const uint64_t w1 = w0 + LINE_WORDS < words ? w0 + LINE_WORDS : words;
        for (uint64_t w = w0; w < w1; ++w)
            any |= unk[w];
    }
    const unsigned long long bits = __ballot(any != 0u);
    if ((threadIdx.x & 63u) == 0u && line < nlines)
        lines[line / 64] = bits;
}

}  // namespace

hipError_t launch_unknown_lines(const uint32_t *unk, uint64_t words, unsigned long long *lines,
                                hipStream_t s)
{
    const uint64_t nlines = (words + LINE_WORDS - 1) / LINE_WORDS;
    if (nlines == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_unknown_lines, dim3((uint32_t)((nlines + 255) / 256)), dim3(256), 0, s,
                       unk, words, lines);
    return hipGetLastError();
}

hipError_t launch_unpack_reference(const uint32_t *packed, uint64_t first, uint64_t n,
                                   uint32_t layout, uint2 *planes, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    const uint64_t nwords = (n + 31) / 32;
    const dim3 grid((uint32_t)((nwords + 255) / 256));
    if (layout == GK_READS_SPLIT)
        hipLaunchKernelGGL(k_unpack_reference<GK_READS_SPLIT>, grid, dim3(256), 0, s, packed,
                           first, n, planes);
    else
        hipLaunchKernelGGL(k_unpack_reference<GK_READS_INTERLEAVED>, grid, dim3(256), 0, s,
                           packed, first, n, planes);
    return hipGetLastError();
}

hipError_t launch_mark_runs(const uint64_t *runs, uint64_t n_runs, uint32_t *unk, hipStream_t s)
{
    if (n_runs == 0)
        return hipSuccess;
    const uint32_t blocks = (uint32_t)(n_runs < 65536 ? n_runs : 65536);
    hipLaunchKernelGGL(k_mark_runs, dim3(blocks), dim3(256), 0, s, runs, n_runs, unk);
    return hipGetLastError();
}

hipError_t launch_count_unknown(const uint32_t *unk, uint64_t words, unsigned long long *counter,
                                hipStream_t s)
{
    if (words == 0)
        return hipSuccess;
    const uint64_t want = (words + 255) / 256;
    const uint32_t blocks = (uint32_t)(want < 16384 ? want : 16384);
    hipLaunchKernelGGL(k_count_unknown, dim3(blocks), dim3(256), 0, s, unk, words, counter);
    return hipGetLastError();
}

}  // namespace gkd

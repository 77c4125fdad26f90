// Calibration kernels for the roofline (measurement support, not part of the
// filter): the device's issue rate of the 32-bit bit-logic VALU instructions
// the filter is made of, and its plain device-to-device copy rate.  Built into
// libgk_calib.so, separate from libgk.so.
//
// VALU rate: every lane runs 8 independent dependency chains of one
// instruction kind, 8 steps per chain per loop iteration (64 instructions),
// written as inline assembly so that the compiler can neither fold nor
// reorder them; a grid of blocks_per_cu * CUs workgroups of 256 lanes.
//   kind 0  v_bfi_b32       (3-input bit select: the amendment's merges)
//   kind 1  v_alignbit_b32  (funnel shift: the window and mask shifts)
//   kind 2  v_xor_b32       (2-input logic: the comparisons)
//   kind 3  v_and_or_b32    (3-input logic)
//   kind 4  v_or3_b32       (3-input logic)
//   kind 5  v_bitop3_b32    (any 3-input logic function; here xor3)
//   kind 6  v_and_b32       (2-input logic, 32-bit VOP2 encoding)
//   kind 7  v_lshlrev_b32   (shift, VOP2 encoding)
//   kind 8  v_xor_b32_e64   (2-input logic in the 64-bit VOP3 encoding)
//   kind 9  v_add_u32       (32-bit add, VOP2 encoding)
//   kind 10 v_perm_b32      (byte permute, 3 inputs)
//   kind 11 v_bcnt_u32_b32  (population count, VOP3 encoding)
// Lane-ops/s = workgroups * 256 * iterations * 64 / kernel time.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

#define GKC_STEP3(OP, x, y, z) asm volatile(OP " %0, %1, %2, %0" : "+v"(x) : "v"(y), "v"(z))
#define GKC_STEP2(OP, x, y) asm volatile(OP " %0, %1, %0" : "+v"(x) : "v"(y))

template <int KIND>
__device__ __forceinline__ void step(uint32_t &x, uint32_t y, uint32_t z)
{
    if (KIND == 0)
        GKC_STEP3("v_bfi_b32", x, y, z);
    else if (KIND == 1)
        GKC_STEP3("v_alignbit_b32", x, y, z);
    else if (KIND == 2)
        GKC_STEP2("v_xor_b32", x, y);
    else if (KIND == 3)
        GKC_STEP3("v_and_or_b32", x, y, z);
    else if (KIND == 4)
        GKC_STEP3("v_or3_b32", x, y, z);
    else if (KIND == 5)
        asm volatile("v_bitop3_b32 %0, %1, %2, %0 bitop3:0x96" : "+v"(x) : "v"(y), "v"(z));
    else if (KIND == 6)
        GKC_STEP2("v_and_b32", x, y);
    else if (KIND == 7)
        GKC_STEP2("v_lshlrev_b32", x, y);
    else if (KIND == 8)
        GKC_STEP2("v_xor_b32_e64", x, y);
    else if (KIND == 9)
        GKC_STEP2("v_add_u32", x, y);
    else if (KIND == 10)
        GKC_STEP3("v_perm_b32", x, y, z);
    else
        GKC_STEP2("v_bcnt_u32_b32", x, y);
}

template <int KIND>
__global__ __launch_bounds__(256) void k_valu_rate(uint32_t iters, uint32_t seed, uint32_t *sink)
{
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    uint32_t a0 = seed ^ (t * 0x9E3779B9u), a1 = a0 * 3u + 1u, a2 = a1 * 5u + 7u,
             a3 = a2 * 9u + 3u, a4 = a3 * 17u + 11u, a5 = a4 * 33u + 5u, a6 = a5 * 65u + 13u,
             a7 = a6 * 129u + 17u;
    const uint32_t y = seed * 0x85EBCA6Bu + t, z = (seed ^ 0xC2B2AE35u) + 3u * t;
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            step<KIND>(a0, y, z);
            step<KIND>(a1, y, z);
            step<KIND>(a2, y, z);
            step<KIND>(a3, y, z);
            step<KIND>(a4, y, z);
            step<KIND>(a5, y, z);
            step<KIND>(a6, y, z);
            step<KIND>(a7, y, z);
        }
    }
    const uint32_t x = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
    if (x == 0x5EEDF00Du)         // keeps the chains live; practically never true
        sink[blockIdx.x] = x;
}

// Plain copy: n16 16-byte words from src to dst, grid-stride.
__global__ __launch_bounds__(256) void k_copy(const uint4 *src, uint4 *dst, uint64_t n16)
{
    const uint64_t stride = (uint64_t)gridDim.x * 256u;
    for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

template <int KIND>
hipError_t launch_valu(uint32_t blocks, uint32_t iters, uint32_t *sink, hipStream_t s)
{
    hipLaunchKernelGGL(k_valu_rate<KIND>, dim3(blocks), dim3(256), 0, s, iters, 0x1234567u, sink);
    return hipGetLastError();
}

hipError_t launch_kind(int kind, uint32_t blocks, uint32_t iters, uint32_t *sink, hipStream_t s)
{
    switch (kind) {
    case 0:
        return launch_valu<0>(blocks, iters, sink, s);
    case 1:
        return launch_valu<1>(blocks, iters, sink, s);
    case 2:
        return launch_valu<2>(blocks, iters, sink, s);
    case 3:
        return launch_valu<3>(blocks, iters, sink, s);
    case 4:
        return launch_valu<4>(blocks, iters, sink, s);
    case 5:
        return launch_valu<5>(blocks, iters, sink, s);
    case 6:
        return launch_valu<6>(blocks, iters, sink, s);
    case 7:
        return launch_valu<7>(blocks, iters, sink, s);
    case 8:
        return launch_valu<8>(blocks, iters, sink, s);
    case 9:
        return launch_valu<9>(blocks, iters, sink, s);
    case 10:
        return launch_valu<10>(blocks, iters, sink, s);
    default:
        return launch_valu<11>(blocks, iters, sink, s);
    }
}

}  // namespace

extern "C" {

// Issue rate of VALU instruction `kind` (0..11, above) on the current device:
// lane-ops per second over `reps` timed launches (after one warm-up), each of
// blocks_per_cu * CUs workgroups running `iters` loop iterations.  *best_ms:
// the fastest launch, from which *lane_ops_per_s is computed.  Returns 0, or
// a negative HIP error code.
int gkc_valu_rate(int kind, uint32_t blocks_per_cu, uint32_t iters, uint32_t reps,
                  double *lane_ops_per_s, double *best_ms)
{
    if (kind < 0 || kind > 11 || blocks_per_cu < 1 || iters < 1 || reps < 1 || !lane_ops_per_s ||
        !best_ms)
        return -1;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess)
        return -(int)e;
    const uint32_t blocks = blocks_per_cu * (uint32_t)cus;
    uint32_t *sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if ((e = hipMalloc(&sink, blocks * sizeof(uint32_t))) != hipSuccess)
        return -(int)e;
    e = hipEventCreate(&e0);
    if (e == hipSuccess)
        e = hipEventCreate(&e1);
    float best = -1.f;
    for (uint32_t r = 0; r <= reps && e == hipSuccess; ++r) {
        e = hipEventRecord(e0, nullptr);
        if (e == hipSuccess)
            e = launch_kind(kind, blocks, iters, sink, nullptr);
        if (e == hipSuccess)
            e = hipEventRecord(e1, nullptr);
        if (e == hipSuccess)
            e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && r > 0 && (best < 0.f || ms < best))
            best = ms;
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    if (e != hipSuccess)
        return -(int)e;
    *best_ms = best;
    *lane_ops_per_s = (double)blocks * 256.0 * (double)iters * 64.0 / (best * 1e-3);
    return 0;
}

// Device-to-device copy rate: bytes read plus bytes written per second for a
// copy of `bytes` (rounded down to 16 B), best of `reps` launches after one
// warm-up, with a grid of 8 workgroups per CU.  Returns 0 or a negative HIP
// error code.
int gkc_copy_rate(uint64_t bytes, uint32_t reps, double *bytes_per_s, double *best_ms)
{
    if (bytes < 16 || reps < 1 || !bytes_per_s || !best_ms)
        return -1;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess)
        return -(int)e;
    const uint64_t n16 = bytes / 16;
    uint4 *src = nullptr, *dst = nullptr;
    if ((e = hipMalloc(&src, n16 * 16)) != hipSuccess)
        return -(int)e;
    if ((e = hipMalloc(&dst, n16 * 16)) != hipSuccess) {
        (void)hipFree(src);
        return -(int)e;
    }
    e = hipMemset(src, 0x5A, n16 * 16);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess)
        e = hipEventCreate(&e0);
    if (e == hipSuccess)
        e = hipEventCreate(&e1);
    float best = -1.f;
    for (uint32_t r = 0; r <= reps && e == hipSuccess; ++r) {
        e = hipEventRecord(e0, nullptr);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_copy, dim3(8u * (uint32_t)cus), dim3(256), 0, nullptr, src, dst,
                               n16);
            e = hipGetLastError();
        }
        if (e == hipSuccess)
            e = hipEventRecord(e1, nullptr);
        if (e == hipSuccess)
            e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && r > 0 && (best < 0.f || ms < best))
            best = ms;
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    (void)hipFree(src);
    (void)hipFree(dst);
    if (e != hipSuccess)
        return -(int)e;
    *best_ms = best;
    *bytes_per_s = 2.0 * (double)(n16 * 16) / (best * 1e-3);
    return 0;
}

}  // extern "C"

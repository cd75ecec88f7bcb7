// Stage 2: inclusive prefix sum of the per-Gaussian tile counts
// (Speedy-Splat Sec. 3.2.2, "InclusiveSum"), taken in depth order: the depth
// order stage leaves order_counts[j] = counts[order[j]], entry j of the scan
// sums order_counts[j'] for j' <= j, so Gaussian order[j] writes its pairs at
// [offsets[j] - order_counts[j], offsets[j]) and the emitted pairs come out
// sorted by depth.
//
// Reduce-then-scan in two launches, so no workgroup ever waits on another:
//   1. each workgroup sums its 4096 counts into a 64-bit partial;
//   2. each workgroup sums the partials of the workgroups before it (a few
//      hundred 8-byte reads from L2), rescans its counts (wave prefix sums,
//      wave totals through LDS) and writes uint32 offsets; the last one writes
//      the grand total P to scan_tmp[0].
// scan_tmp layout: [0] = P, [1 + b] = the partial of block b.
#include "ss_internal.h"

namespace ss {
namespace {

constexpr int kBlock = 256;
constexpr int kItems = 16;                       // counts per lane
constexpr int kPerBlock = kBlock * kItems;       // 4096

__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t x) {
    const int lane = (int)__lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

__global__ __launch_bounds__(kBlock) void k_block_sums(const uint32_t* __restrict__ counts,
                                                       int64_t n, uint64_t* __restrict__ tmp,
                                                       const uint64_t* __restrict__ totals) {
    n = (int64_t)frame_count(totals, 1, (uint64_t)n);
    const int64_t base = (int64_t)blockIdx.x * kPerBlock;
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
        if (i < n) s += counts[i];
    }
    s = wave_incl_scan(s);
    __shared__ uint64_t wsum[kBlock / 64];
    if (__lane_id() == 63) wsum[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < kBlock / 64; ++w) t += wsum[w];
        tmp[1 + blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_block_scan(const uint32_t* __restrict__ counts,
                                                       int64_t n, uint64_t* __restrict__ tmp,
                                                       uint32_t* __restrict__ offsets,
                                                       const uint64_t* __restrict__ totals) {
    n = (int64_t)frame_count(totals, 1, (uint64_t)n);
    // this block's offset: the partials of the blocks before it
    __shared__ uint64_t osum[kBlock / 64];
    uint64_t o = 0;
    for (int64_t k = threadIdx.x; k < (int64_t)blockIdx.x; k += kBlock) o += tmp[1 + k];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) o += __shfl_xor(o, d, 64);
    if (__lane_id() == 0) osum[threadIdx.x >> 6] = o;
    // Lane l of the workgroup owns entries [base + l*16, base + l*16 + 16).
    const int64_t base = (int64_t)blockIdx.x * kPerBlock;
    const int64_t first = base + (int64_t)threadIdx.x * kItems;
    uint32_t c[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) c[k] = (first + k < n) ? counts[first + k] : 0u;
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) s += c[k];
    const uint64_t inc = wave_incl_scan(s);
    __shared__ uint64_t wsum[kBlock / 64];
    const int w = threadIdx.x >> 6;
    if (__lane_id() == 63) wsum[w] = inc;
    __syncthreads();
    uint64_t run = inc - s;
#pragma unroll
    for (int k = 0; k < kBlock / 64; ++k) run += osum[k] + (k < w ? wsum[k] : 0u);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        run += c[k];
        if (first + k < n) offsets[first + k] = (uint32_t)run;
    }
    if (blockIdx.x + 1 == gridDim.x && threadIdx.x + 1 == kBlock) tmp[0] = run;
}

}  // namespace

int64_t scan_tmp_words(int64_t n) { return 1 + (n + kPerBlock - 1) / kPerBlock; }

hipError_t launch_scan(int64_t n, const ss_frame& f, hipStream_t s, const uint64_t* totals) {
    const int64_t nb = (n + kPerBlock - 1) / kPerBlock;
    if (nb > 0) {
        hipLaunchKernelGGL(k_block_sums, dim3((unsigned)nb), dim3(kBlock), 0, s,
                           f.order_counts, n, f.scan_tmp, totals);
    }
    // one workgroup when n == 0, to write P = 0
    hipLaunchKernelGGL(k_block_scan, dim3((unsigned)(nb > 0 ? nb : 1)), dim3(kBlock), 0, s,
                       f.order_counts, n, f.scan_tmp, f.offsets, totals);
    return hipGetLastError();
}

}  // namespace ss

// Stage 2: inclusive prefix sum of the per-Gaussian tile counts
// (Speedy-Splat Sec. 3.2.2, "InclusiveSum"), taken in depth order: the depth
// order stage leaves order_counts[j] = counts[order[j]], entry j of the scan
// sums order_counts[j'] for j' <= j, so Gaussian order[j] writes its pairs at
// [offsets[j] - order_counts[j], offsets[j]) and the emitted pairs come out
// sorted by depth.
//
// Reduce-then-scan in three launches, so no workgroup ever waits on another:
//   1. each workgroup sums its 4096 counts into a 64-bit partial;
//   2. one workgroup turns the partials into exclusive 64-bit block offsets
//      and writes the grand total P to scan_tmp[0];
//   3. each workgroup rescans its counts (wave prefix sums with DPP-backed
//      shuffles, wave totals through LDS) and writes uint32 offsets.
// scan_tmp layout: [0] = P, [1 + b] = exclusive offset of block b.
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
                                                       int64_t n, uint64_t* __restrict__ tmp) {
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

// One workgroup of 1024 lanes: exclusive scan of nb partials in place.
__global__ __launch_bounds__(1024) void k_scan_partials(uint64_t* __restrict__ tmp, int64_t nb) {
    __shared__ uint64_t wsum[16];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const uint64_t x = i < nb ? tmp[1 + i] : 0;
        uint64_t inc = wave_incl_scan(x);
        const int w = threadIdx.x >> 6;
        if (__lane_id() == 63) wsum[w] = inc;
        __syncthreads();
        uint64_t before = carry;
        for (int k = 0; k < w; ++k) before += wsum[k];
        if (i < nb) tmp[1 + i] = before + inc - x;
        __syncthreads();
        if (threadIdx.x == 1023) carry = before + inc;
        __syncthreads();
    }
    if (threadIdx.x == 0) tmp[0] = carry;
}

__global__ __launch_bounds__(kBlock) void k_block_scan(const uint32_t* __restrict__ counts,
                                                       int64_t n, const uint64_t* __restrict__ tmp,
                                                       uint32_t* __restrict__ offsets) {
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
    uint64_t run = tmp[1 + blockIdx.x] + inc - s;
    for (int k = 0; k < w; ++k) run += wsum[k];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        run += c[k];
        if (first + k < n) offsets[first + k] = (uint32_t)run;
    }
}

}  // namespace

int64_t scan_tmp_words(int64_t n) { return 1 + (n + kPerBlock - 1) / kPerBlock; }

hipError_t launch_scan(int64_t n, const ss_frame& f, hipStream_t s) {
    const int64_t nb = (n + kPerBlock - 1) / kPerBlock;
    if (nb > 0) {
        hipLaunchKernelGGL(k_block_sums, dim3((unsigned)nb), dim3(kBlock), 0, s,
                           f.order_counts, n, f.scan_tmp);
    }
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, f.scan_tmp, nb);
    if (nb > 0) {
        hipLaunchKernelGGL(k_block_scan, dim3((unsigned)nb), dim3(kBlock), 0, s,
                           f.order_counts, n, f.scan_tmp, f.offsets);
    }
    return hipGetLastError();
}

}  // namespace ss

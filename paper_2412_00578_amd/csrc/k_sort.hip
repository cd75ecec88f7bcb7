// Stage 4: LSD radix sort of the (tile | depth) keys with their Gaussian
// indices (Speedy-Splat Sec. 3.2 "RadixSort"), and stage 5: per-tile ranges
// ("identifyTileRanges").
//
// Only the low 32 + ceil(log2(n_tiles)) key bits can be non-zero, so the sort
// runs ceil(bits / 8) passes of 8-bit digits.  Each pass is reduce-then-scan:
//   hist     workgroup b counts the digits of its contiguous key chunk
//   scan     one workgroup turns the (digit, workgroup) counts, digit-major,
//            into exclusive output offsets
//   scatter  workgroup b re-reads its chunk in 4096-key sub-tiles; each wave
//            ranks 64 keys at a time by matching digits with 8 ballots
//            (stable: lane order), keeps per-wave running digit counts in LDS,
//            and writes each key at offset(digit, b) + keys of that digit
//            before it in the chunk.
// No workgroup waits on another, so there is no forward-progress assumption.
#include "ss_internal.h"

namespace ss {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kItems = 16;                    // keys per lane per sub-tile
constexpr int kSub = kBlock * kItems;         // 4096 keys
constexpr int kRadix = 256;
constexpr int kMaxGrid = 1024;

struct Plan {
    uint32_t grid;        // workgroups
    uint64_t chunk;       // keys per workgroup (multiple of kSub)
};

Plan make_plan(uint64_t n) {
    const uint64_t subs = (n + kSub - 1) / kSub;
    uint64_t g = subs < (uint64_t)kMaxGrid ? subs : (uint64_t)kMaxGrid;
    if (g == 0) g = 1;
    const uint64_t per = (subs + g - 1) / g;
    const uint64_t grid = per ? (subs + per - 1) / per : 1;
    return Plan{(uint32_t)(grid ? grid : 1), (per ? per : 1) * kSub};
}

__global__ __launch_bounds__(kBlock) void k_hist(const uint64_t* __restrict__ keys, uint64_t n,
                                                 int shift, uint64_t chunk, uint32_t grid,
                                                 uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[kWaves][kRadix];
    for (int k = threadIdx.x; k < kWaves * kRadix; k += kBlock) (&h[0][0])[k] = 0u;
    __syncthreads();
    const uint64_t lo = (uint64_t)blockIdx.x * chunk;
    const uint64_t hi = lo + chunk < n ? lo + chunk : n;
    const int w = threadIdx.x >> 6;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
        const uint32_t d = (uint32_t)(keys[i] >> shift) & (kRadix - 1);
        atomicAdd(&h[w][d], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kRadix; d += kBlock) {
        uint32_t s = 0;
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww) s += h[ww][d];
        hist[(uint64_t)d * grid + blockIdx.x] = s;
    }
}

__device__ __forceinline__ uint32_t wave_incl_scan32(uint32_t x) {
    const int lane = (int)__lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive scan of m = 256 * grid counts in place; one workgroup of 1024.
__global__ __launch_bounds__(1024) void k_hist_scan(uint32_t* __restrict__ hist, uint32_t m) {
    __shared__ uint32_t wsum[16];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    constexpr int kPer = 4;
    for (uint32_t base = 0; base < m; base += 1024 * kPer) {
        const uint32_t first = base + threadIdx.x * kPer;
        uint32_t c[kPer];
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            c[k] = first + k < m ? hist[first + k] : 0u;
            s += c[k];
        }
        const uint32_t inc = wave_incl_scan32(s);
        const int w = threadIdx.x >> 6;
        if (__lane_id() == 63) wsum[w] = inc;
        __syncthreads();
        uint32_t run = carry + inc - s;
        for (int k = 0; k < w; ++k) run += wsum[k];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            if (first + k < m) hist[first + k] = run;
            run += c[k];
        }
        __syncthreads();
        if (threadIdx.x == 1023) carry = run;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_scatter(const uint64_t* __restrict__ keys_in,
                                                    const uint32_t* __restrict__ vals_in,
                                                    uint64_t* __restrict__ keys_out,
                                                    uint32_t* __restrict__ vals_out, uint64_t n,
                                                    int shift, uint64_t chunk, uint32_t grid,
                                                    const uint32_t* __restrict__ hist) {
    __shared__ uint32_t base[kRadix];
    __shared__ uint32_t wcnt[kWaves][kRadix];
    __shared__ uint32_t tot[kRadix];
    for (int d = threadIdx.x; d < kRadix; d += kBlock) base[d] = hist[(uint64_t)d * grid + blockIdx.x];
    const uint64_t lo = (uint64_t)blockIdx.x * chunk;
    const uint64_t hi = lo + chunk < n ? lo + chunk : n;
    const int w = threadIdx.x >> 6;
    const unsigned lane = __lane_id();
    for (uint64_t sub = lo; sub < hi; sub += kSub) {
        for (int k = threadIdx.x; k < kWaves * kRadix; k += kBlock) (&wcnt[0][0])[k] = 0u;
        __syncthreads();
        uint64_t key[kItems];
        uint32_t val[kItems];
        uint32_t rank[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const uint64_t idx = sub + (uint64_t)w * (64 * kItems) + (uint64_t)k * 64 + lane;
            const bool valid = idx < hi;
            key[k] = valid ? keys_in[idx] : 0ull;
            val[k] = valid ? vals_in[idx] : 0u;
            const uint32_t d = (uint32_t)(key[k] >> shift) & (kRadix - 1);
            uint64_t m = __ballot(valid);
#pragma unroll
            for (int bit = 0; bit < 8; ++bit) {
                const bool set = (d >> bit) & 1u;
                const uint64_t bb = __ballot(set);
                m &= set ? bb : ~bb;
            }
            const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            const uint32_t pre = wcnt[w][d];
            rank[k] = pre + below;
            if (valid && below == 0u) wcnt[w][d] = pre + (uint32_t)__popcll(m);
        }
        __syncthreads();
        for (int d = threadIdx.x; d < kRadix; d += kBlock) {
            uint32_t s = 0;
#pragma unroll
            for (int ww = 0; ww < kWaves; ++ww) {
                const uint32_t c = wcnt[ww][d];
                wcnt[ww][d] = s;
                s += c;
            }
            tot[d] = s;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const uint64_t idx = sub + (uint64_t)w * (64 * kItems) + (uint64_t)k * 64 + lane;
            if (idx < hi) {
                const uint32_t d = (uint32_t)(key[k] >> shift) & (kRadix - 1);
                const uint32_t pos = base[d] + wcnt[w][d] + rank[k];
                if (pos < n) {
                    keys_out[pos] = key[k];
                    vals_out[pos] = val[k];
                }
            }
        }
        __syncthreads();
        for (int d = threadIdx.x; d < kRadix; d += kBlock) base[d] += tot[d];
        __syncthreads();
    }
}

// One lane per boundary position i in [0, n]: every tile whose run starts at i
// gets start = i, every tile whose run ends at i gets end = i.
__global__ __launch_bounds__(256) void k_ranges(const uint64_t* __restrict__ keys, uint64_t n,
                                                int n_tiles, uint32_t* __restrict__ ranges) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    const int prev = i == 0 ? -1 : (int)(keys[i - 1] >> 32);
    const int cur = i == n ? n_tiles : (int)(keys[i] >> 32);
    if (prev == cur) return;
    for (int t = prev + 1; t <= cur && t < n_tiles; ++t) ranges[2 * t] = (uint32_t)i;
    for (int t = prev < 0 ? 0 : prev; t < cur && t < n_tiles; ++t) ranges[2 * t + 1] = (uint32_t)i;
}

}  // namespace

int sort_passes(int bits) { return (bits + 7) / 8; }

int64_t sort_tmp_words(uint64_t) { return (int64_t)kRadix * kMaxGrid; }

hipError_t launch_sort(const ss_pairs& p, int buf, uint64_t n, int bits, int* out_buf,
                       hipStream_t s) {
    int cur = buf;
    if (n > 1) {
        const Plan plan = make_plan(n);
        const int passes = sort_passes(bits);
        for (int pass = 0; pass < passes; ++pass) {
            const int shift = pass * 8;
            hipLaunchKernelGGL(k_hist, dim3(plan.grid), dim3(kBlock), 0, s, p.keys[cur], n, shift,
                               plan.chunk, plan.grid, p.sort_tmp);
            hipLaunchKernelGGL(k_hist_scan, dim3(1), dim3(1024), 0, s, p.sort_tmp,
                               (uint32_t)(kRadix * plan.grid));
            hipLaunchKernelGGL(k_scatter, dim3(plan.grid), dim3(kBlock), 0, s, p.keys[cur],
                               p.values[cur], p.keys[1 - cur], p.values[1 - cur], n, shift,
                               plan.chunk, plan.grid, p.sort_tmp);
            cur = 1 - cur;
        }
    }
    *out_buf = cur;
    return hipGetLastError();
}

hipError_t launch_ranges(const uint64_t* keys, uint64_t n, int n_tiles, uint32_t* ranges,
                         hipStream_t s) {
    const uint64_t items = n + 1;
    const uint64_t grid = (items + 255) / 256;
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)grid), dim3(256), 0, s, keys, n, n_tiles, ranges);
    return hipGetLastError();
}

}  // namespace ss

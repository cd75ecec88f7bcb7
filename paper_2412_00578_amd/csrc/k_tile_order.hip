// The blend's tile work order (launch index -> tile), from the per-tile
// ranges (Speedy-Splat Sec. 3.2.3: one workgroup per tile; the order in which
// the tiles are launched is this implementation's load balancing).
#include "ss_internal.h"

namespace ss {
namespace {

// Tile work order.  Workgroups are dispatched in launch order, round-robin
// over the 8 XCDs (launch index b runs on XCD b mod 8), each XCD with its own
// L2.  Tiles are grouped in 4x4-tile blocks, dealt round-robin over the XCDs
// (neighbouring tiles share Gaussians, so a block's records are fetched into
// one L2), and each XCD runs its tiles longest list first: its long tiles
// start first and short ones fill the gaps behind them, instead of a long
// tile starting late and running on alone at the end of the launch.  List
// lengths are bucketed by 8 entries (tiles of one bucket in no particular
// order).  Launch index x + 8 r holds the r-th tile of XCD x's list; an XCD
// with more tiles than such indices passes its shortest ones to the free
// indices of the others.  One workgroup.
constexpr int kOrderBuckets = 1024;
constexpr int kOrderKeys = 8 * kOrderBuckets;     // (XCD, bucket) pairs
constexpr int kOrderThreads = 1024;
constexpr int kOrderPer = kOrderKeys / kOrderThreads;

// XCD-major, longest bucket first within an XCD.  tx_single: the tile grid
// width when the batch has one item (whose tiles start at 0).
__device__ __forceinline__ uint32_t order_key(const Item* __restrict__ items, int n_items,
                                              int tx_single, const uint32_t* __restrict__ ranges,
                                              int t) {
    int k = 0, tx_n = tx_single, lt = t;
    if (n_items != 1) {
        k = item_of_tile(items, n_items, t);
        tx_n = items[k].tx_n;
        lt = t - items[k].tile_off;
    }
    const int bx = (lt % tx_n) >> 2, by = (lt / tx_n) >> 2;
    const uint32_t x = (uint32_t)(by * ((tx_n + 3) >> 2) + bx + 3 * k) & 7u;
    const uint2 r = *reinterpret_cast<const uint2*>(ranges + 2 * t);
    const uint32_t len = r.y - r.x;
    const uint32_t b = len >> 3 < (uint32_t)kOrderBuckets - 1u ? len >> 3
                                                               : (uint32_t)kOrderBuckets - 1u;
    return x * kOrderBuckets + (kOrderBuckets - 1u - b);
}

// counts_out (host memory the device can write, or null) receives the frame
// counts (totals[0], totals[1]).
__global__ __launch_bounds__(kOrderThreads) void k_tile_order(const Item* __restrict__ items,
                                                              BatchDims dims,
                                                              const uint32_t* __restrict__ ranges,
                                                              uint32_t* __restrict__ order,
                                                              uint32_t* __restrict__ queue,
                                                              const uint64_t* __restrict__ totals,
                                                              uint64_t* __restrict__ counts_out) {
    __shared__ uint32_t h[kOrderKeys];
    if (threadIdx.x < 8) queue[threadIdx.x] = 0u;     // the persistent blend's counters
    if (counts_out && threadIdx.x < 2)
        __hip_atomic_store(counts_out + threadIdx.x, totals[threadIdx.x], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
    __shared__ uint32_t s_w[kOrderThreads / 64];
    __shared__ uint32_t s_start[9], s_cap[8], s_over[9], s_free[9];
    const int t0 = (int)threadIdx.x;
    const int n = dims.n_tiles;
    const int tx1 = items[0].tx_n;
#pragma unroll
    for (int u = 0; u < kOrderPer; ++u) h[t0 * kOrderPer + u] = 0u;
    __syncthreads();
    // the keys of the first kOrderPer * 1024 tiles stay in registers for the
    // second pass (their loads are issued together)
    uint32_t kc[kOrderPer];
#pragma unroll
    for (int u = 0; u < kOrderPer; ++u) {
        const int t = t0 + u * kOrderThreads;
        kc[u] = t < n ? order_key(items, dims.n_items, tx1, ranges, t) : 0u;
    }
#pragma unroll
    for (int u = 0; u < kOrderPer; ++u)
        if (t0 + u * kOrderThreads < n) atomicAdd(&h[kc[u]], 1u);
    for (int t = t0 + kOrderPer * kOrderThreads; t < n; t += kOrderThreads)
        atomicAdd(&h[order_key(items, dims.n_items, tx1, ranges, t)], 1u);
    __syncthreads();
    // exclusive scan of the key counts; thread t0 owns keys kOrderPer t0 ..
    uint32_t c[kOrderPer], sum = 0;
#pragma unroll
    for (int u = 0; u < kOrderPer; ++u) {
        c[u] = h[t0 * kOrderPer + u];
        sum += c[u];
    }
    uint32_t incl = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(incl, d, 64);
        if ((t0 & 63) >= d) incl += y;
    }
    if ((t0 & 63) == 63) s_w[t0 >> 6] = incl;
    __syncthreads();
    uint32_t run = incl - sum;
    for (int k = 0; k < (t0 >> 6); ++k) run += s_w[k];
#pragma unroll
    for (int u = 0; u < kOrderPer; ++u) {
        h[t0 * kOrderPer + u] = run;
        run += c[u];
    }
    __syncthreads();
    if (t0 < 8) {
        // XCD t0's list is [s_start[t0], s_start[t0 + 1]) of the sorted keys;
        // launch indices x + 8 r < n number cap_x
        s_start[t0] = h[t0 * kOrderBuckets];
        s_cap[t0] = t0 < n ? (uint32_t)(n - t0 + 7) / 8u : 0u;
        if (t0 == 0) s_start[8] = (uint32_t)n;
    }
    __syncthreads();
    if (t0 == 0) {
        uint32_t over = 0, fr = 0;
        for (int x = 0; x < 8; ++x) {
            const uint32_t len = s_start[x + 1] - s_start[x];
            s_over[x] = over;
            s_free[x] = fr;
            over += len > s_cap[x] ? len - s_cap[x] : 0u;
            fr += s_cap[x] > len ? s_cap[x] - len : 0u;
        }
        s_over[8] = over;
        s_free[8] = fr;
    }
    __syncthreads();
    for (int t = t0; t < n; t += kOrderThreads) {
        const int u = (t - t0) / kOrderThreads;
        const uint32_t key = u < kOrderPer ? kc[u] : order_key(items, dims.n_items, tx1, ranges, t);
        const uint32_t x = key / kOrderBuckets;
        const uint32_t r = atomicAdd(&h[key], 1u) - s_start[x];
        if (r < s_cap[x]) {
            order[x + 8u * r] = (uint32_t)t;
        } else {
            // the o-th overflow tile takes the o-th free launch index
            const uint32_t o = s_over[x] + (r - s_cap[x]);
            uint32_t y = 0;
            while (y < 7u && s_free[y + 1] <= o) ++y;
            const uint32_t leny = s_start[y + 1] - s_start[y];
            order[y + 8u * (leny + (o - s_free[y]))] = (uint32_t)t;
        }
    }
}

}  // namespace

hipError_t launch_tile_order(const Item* items, const BatchDims& d, const ss_frame& f,
                             hipStream_t s, uint64_t* counts_out) {
    if (d.n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(kOrderThreads), 0, s, items, d, f.ranges,
                       tile_order_of(f.table, d.n_items),
                       tile_queue_of(f.table, d.n_items, d.n_tiles), f.totals, counts_out);
    return hipGetLastError();
}

}  // namespace ss

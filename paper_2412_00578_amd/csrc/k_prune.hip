// Pruning by score (Speedy-Splat Sec. 4.2.2 Soft Pruning and Sec. 4.2.3 Hard
// Pruning, with the efficient pruning score of Sec. 4.2.1): keep the n_keep
// Gaussians with the highest scores, ties at the threshold broken in favour of
// the lower index, and compact the resident parameter arrays to them.
//
// Selection is a most-significant-digit radix select on the score's bit
// pattern (scores are sums of squares, so for non-negative floats the bits
// order like the values; NaN and non-positive scores count as 0):
//   4 passes, each: k_sel_hist counts the next 8-bit digit of every key that
//   matches the digits chosen so far (per-wave LDS histograms, one global add
//   per bucket and workgroup), then one workgroup (k_sel_pick) walks the 256
//   buckets from the top to the one holding the k-th largest key and narrows
//   the prefix.  After the last pass the prefix is the threshold key T and the
//   state holds how many keys equal to T are kept.
// Compaction is reduce-then-scan (no workgroup waits on another): k_sel_count
// counts per 4096-key block the keys above T and equal to T; k_sel_write sums
// the counts of the blocks before it, ranks its keys equal to T by index, and
// writes the kept indices in ascending order.  k_gather copies the kept
// Gaussians' rows of every parameter array.
#include "ss_internal.h"

namespace ss {
namespace {

constexpr int kBlock = 256;
constexpr int kItems = 16;
constexpr int kPerBlock = kBlock * kItems;      // keys per compaction block
constexpr int kHistBlock = 256;
constexpr int kHistItems = 16;

// scratch layout (uint32 words): [0, 256) histogram, [256] prefix, [257] keys
// still to take at or below the prefix, then 2 counts per compaction block.
constexpr int kHist = 0, kPrefix = 256, kRemain = 257, kBlocks = 260;

__device__ __forceinline__ uint32_t score_key(float s) {
    return (s > 0.0f) ? __float_as_uint(s) : 0u;   // NaN and s <= 0 fail the test
}

__global__ void k_sel_init(uint32_t* __restrict__ st, uint32_t k) {
    const int t = (int)threadIdx.x;
    st[kHist + t] = 0u;
    if (t == 0) {
        st[kPrefix] = 0u;
        st[kRemain] = k;
    }
}

// Histogram of digit (key >> shift) & 255 over the keys whose bits above
// shift + 8 equal the prefix's.
__global__ __launch_bounds__(kHistBlock) void k_sel_hist(const float* __restrict__ score,
                                                         int64_t n, int shift,
                                                         uint32_t* __restrict__ st) {
    __shared__ uint32_t h[kHistBlock / 64][256];
    for (int k = threadIdx.x; k < (kHistBlock / 64) * 256; k += kHistBlock) (&h[0][0])[k] = 0u;
    __syncthreads();
    const uint32_t prefix = st[kPrefix];
    const int hs = shift + 8;
    const int w = (int)(threadIdx.x >> 6);
    const int64_t base = (int64_t)blockIdx.x * kHistBlock * kHistItems;
#pragma unroll 4
    for (int u = 0; u < kHistItems; ++u) {
        const int64_t i = base + (int64_t)u * kHistBlock + threadIdx.x;
        if (i < n) {
            const uint32_t key = score_key(score[i]);
            const bool match = hs >= 32 || (key >> hs) == (prefix >> hs);
            if (match) atomicAdd(&h[w][(key >> shift) & 255u], 1u);
        }
    }
    __syncthreads();
    const int d = (int)threadIdx.x;
    uint32_t c = 0;
#pragma unroll
    for (int ww = 0; ww < kHistBlock / 64; ++ww) c += h[ww][d];
    if (c) atomicAdd(&st[kHist + d], c);
}

// One workgroup of 256 lanes, lane d holding bucket d: the bucket of the
// k-th largest key (k = the keys still to take), the new prefix, and the
// keys still to take inside that bucket; clears the histogram.
__global__ __launch_bounds__(256) void k_sel_pick(uint32_t* __restrict__ st, int shift) {
    __shared__ uint32_t s_c[256];
    __shared__ uint32_t s_above[256];
    const int d = (int)threadIdx.x;
    const uint32_t c = st[kHist + d];
    s_c[d] = c;
    __syncthreads();
    // keys in buckets above d (a plain loop: one workgroup, once per pass)
    uint32_t above = 0;
    for (int e = d + 1; e < 256; ++e) above += s_c[e];
    s_above[d] = above;
    __syncthreads();
    const uint32_t rem = st[kRemain];
    __syncthreads();
    if (c > 0 && above < rem && rem <= above + c) {     // exactly one bucket
        st[kPrefix] = st[kPrefix] | ((uint32_t)d << shift);
        st[kRemain] = rem - above;
    }
    st[kHist + d] = 0u;
}

__device__ __forceinline__ uint32_t block_sum(uint32_t x, uint32_t* wsum) {
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    if (__lane_id() == 0) wsum[threadIdx.x >> 6] = x;
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) t += wsum[w];
    __syncthreads();
    return t;
}

// Per block: keys above the threshold and keys equal to it.
__global__ __launch_bounds__(kBlock) void k_sel_count(const float* __restrict__ score, int64_t n,
                                                      uint32_t* __restrict__ st) {
    __shared__ uint32_t wsum[kBlock / 64];
    const uint32_t T = st[kPrefix];
    const int64_t base = (int64_t)blockIdx.x * kPerBlock;
    uint32_t gt = 0, eq = 0;
#pragma unroll 4
    for (int u = 0; u < kItems; ++u) {
        const int64_t i = base + (int64_t)u * kBlock + threadIdx.x;
        if (i < n) {
            const uint32_t key = score_key(score[i]);
            gt += key > T;
            eq += key == T;
        }
    }
    gt = block_sum(gt, wsum);
    eq = block_sum(eq, wsum);
    if (threadIdx.x == 0) {
        st[kBlocks + 2 * blockIdx.x] = gt;
        st[kBlocks + 2 * blockIdx.x + 1] = eq;
    }
}

// Exclusive prefix over the block's lanes in index order: each lane holds
// kItems consecutive keys.
__device__ __forceinline__ uint32_t block_excl(uint32_t x, uint32_t* wsum) {
    const int lane = (int)__lane_id();
    uint32_t incl = x;
    for (int dd = 1; dd < 64; dd <<= 1) {
        const uint32_t y = __shfl_up(incl, dd, 64);
        if (lane >= dd) incl += y;
    }
    if (lane == 63) wsum[threadIdx.x >> 6] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) before += wsum[w];
    __syncthreads();
    return before + incl - x;
}

// Kept keys: those above T, and the first `remain` keys equal to T in index
// order; written in ascending index order.
__global__ __launch_bounds__(kBlock) void k_sel_write(const float* __restrict__ score, int64_t n,
                                                      const uint32_t* __restrict__ st,
                                                      uint32_t* __restrict__ keep_idx) {
    __shared__ uint32_t s_gt[kBlock / 64], s_eq[kBlock / 64], wsum[kBlock / 64];
    const uint32_t T = st[kPrefix], take_eq = st[kRemain];
    uint32_t gt0 = 0, eq0 = 0;
    for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += kBlock) {
        gt0 += st[kBlocks + 2 * b];
        eq0 += st[kBlocks + 2 * b + 1];
    }
    for (int m = 32; m >= 1; m >>= 1) {
        gt0 += __shfl_xor(gt0, m, 64);
        eq0 += __shfl_xor(eq0, m, 64);
    }
    if (__lane_id() == 0) {
        s_gt[threadIdx.x >> 6] = gt0;
        s_eq[threadIdx.x >> 6] = eq0;
    }
    __syncthreads();
    gt0 = eq0 = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        gt0 += s_gt[w];
        eq0 += s_eq[w];
    }
    // lane t holds keys base + kItems t .. base + kItems t + kItems - 1
    const int64_t first = (int64_t)blockIdx.x * kPerBlock + (int64_t)threadIdx.x * kItems;
    uint32_t key[kItems];
    uint32_t my_eq = 0;
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        const int64_t i = first + u;
        key[u] = i < n ? score_key(score[i]) : 0u;
        my_eq += (i < n && key[u] == T) ? 1u : 0u;
    }
    uint32_t eq_rank = eq0 + block_excl(my_eq, wsum);
    uint32_t my_keep = 0;
    uint32_t r = eq_rank;
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        const int64_t i = first + u;
        const bool eq = i < n && key[u] == T;
        const bool keep = i < n && (key[u] > T || (eq && r < take_eq));
        r += eq ? 1u : 0u;
        my_keep += keep ? 1u : 0u;
    }
    // kept before this block: every key above T, and the keys equal to T
    // there up to take_eq
    const uint32_t kept0 = gt0 + (eq0 < take_eq ? eq0 : take_eq);
    uint32_t pos = kept0 + block_excl(my_keep, wsum);
    r = eq_rank;
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        const int64_t i = first + u;
        const bool eq = i < n && key[u] == T;
        const bool keep = i < n && (key[u] > T || (eq && r < take_eq));
        r += eq ? 1u : 0u;
        if (keep) keep_idx[pos++] = (uint32_t)i;
    }
}

// dst[j * w + c] = src[idx[j] * w + c] for j < m, c < w.
__global__ __launch_bounds__(256) void k_gather(const float* __restrict__ src,
                                                const uint32_t* __restrict__ idx, int64_t m,
                                                int w, float* __restrict__ dst) {
    const int64_t total = m * (int64_t)w;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = e / w;
        const int c = (int)(e - j * w);
        dst[e] = src[(int64_t)idx[j] * w + c];
    }
}

unsigned gather_grid(int64_t total) {
    const int64_t g = (total + 255) / 256;
    return (unsigned)(g < 8192 ? (g > 0 ? g : 1) : 8192);
}

}  // namespace

int64_t prune_tmp_words(int64_t n) {
    return kBlocks + 2 * ((n + kPerBlock - 1) / kPerBlock);
}

hipError_t launch_prune_select(const float* score, int64_t n, int64_t n_keep, uint32_t* keep_idx,
                               uint32_t* tmp, hipStream_t s) {
    if (n_keep <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, tmp, (uint32_t)n_keep);
    const unsigned hgrid = (unsigned)((n + kHistBlock * kHistItems - 1) / (kHistBlock * kHistItems));
    for (int shift = 24; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(k_sel_hist, dim3(hgrid), dim3(kHistBlock), 0, s, score, n, shift, tmp);
        hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(256), 0, s, tmp, shift);
    }
    const unsigned grid = (unsigned)((n + kPerBlock - 1) / kPerBlock);
    hipLaunchKernelGGL(k_sel_count, dim3(grid), dim3(kBlock), 0, s, score, n, tmp);
    hipLaunchKernelGGL(k_sel_write, dim3(grid), dim3(kBlock), 0, s, score, n, tmp, keep_idx);
    return hipGetLastError();
}

hipError_t launch_gather(const float* src, const uint32_t* idx, int64_t m, int w, float* dst,
                         hipStream_t s) {
    if (m <= 0 || w <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(gather_grid(m * (int64_t)w)), dim3(256), 0, s, src, idx, m,
                       w, dst);
    return hipGetLastError();
}

}  // namespace ss

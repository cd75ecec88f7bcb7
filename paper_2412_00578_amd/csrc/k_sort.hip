// The sorts of the pipeline (Speedy-Splat Sec. 3.2.2, "RadixSort") and stage 5,
// per-tile ranges ("identifyTileRanges").
//
// The paper sorts the pairs once on the 64-bit key tile << 32 | bits(depth).
// The same order (tile, then depth, then Gaussian index) comes from two
// shorter stable sorts:
//   depth order  the record slots by bits(depth) (culled slots last), 4 passes
//                over n slots;
//   tile sort    the pairs, emitted in depth order, by tile id alone:
//                ceil(log2(n_tiles)) bits, 2 passes at 1600x1040,
// which moves about a third of the bytes of six passes over 12-byte pairs.
//
// Both are LSD radix sorts with digits of at most 8 bits, the key bits split
// evenly over the passes (the tile sort's 13 bits as 6 + 7).  Each pass is
// reduce-then-scan, so no workgroup ever waits on another:
//   hist     workgroup b counts the digits of its contiguous key chunk
//   dscan    256 workgroups, one per digit: exclusive scan of that digit's
//            per-workgroup counts, and the digit's total
//   scatter  workgroup b turns the digit totals into digit starts, re-reads its
//            chunk in 2048-key (or, for short sorts, 1024-key) sub-tiles, ranks
//            each key stably (each wave
//            matches 64 digits at a time with 8 ballots; per-wave running
//            counts live in LDS), reorders the sub-tile by digit in LDS and
//            writes every digit run to its global offset with consecutive
//            lanes on consecutive addresses.
#include <mutex>

#include "ss_internal.h"

namespace ss {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kItemsLarge = 8;                // keys per lane per sub-tile: 2048 keys
constexpr int kItemsSmall = 4;                // 1024 keys, for sorts of < 512k keys
constexpr int kRadix = 256;
constexpr int kMaxGrid = 1024;

struct Plan {
    uint32_t grid;        // workgroups
    uint64_t chunk;       // keys per workgroup (multiple of the sub-tile)
    int items;            // keys per lane per sub-tile
};

// Sub-tiles of 2048 keys, or of 1024 for short sorts (fewer than 128 x 4096
// keys), where larger sub-tiles would leave CUs idle.
Plan make_plan(uint64_t n) {
    const int items = (n + 4095) / 4096 < 128 ? kItemsSmall : kItemsLarge;
    const uint64_t kSub = (uint64_t)kBlock * items;
    const uint64_t subs = (n + kSub - 1) / kSub;
    uint64_t g = subs < (uint64_t)kMaxGrid ? subs : (uint64_t)kMaxGrid;
    if (g == 0) g = 1;
    const uint64_t per = (subs + g - 1) / g;
    const uint64_t grid = per ? (subs + per - 1) / per : 1;
    return Plan{(uint32_t)(grid ? grid : 1), (per ? per : 1) * kSub, items};
}

template <class K>
__device__ __forceinline__ uint32_t digit_of(K key, int shift, uint32_t dmask) {
    return (uint32_t)(key >> shift) & dmask;
}

// Keys this pass reads and each workgroup's chunk.  With device frame counts
// the grid was planned for the bound n and the chunk is re-planned for the
// count: the same sub-tiles spread over the same grid, every workgroup of
// k_hist and k_scatter computing the same chunk.
__device__ __forceinline__ void pass_extent(const uint64_t* totals, int word, uint64_t sub,
                                            uint32_t grid, uint64_t& n, uint64_t& chunk) {
    if (!totals) return;
    n = frame_count(totals, word, n);
    const uint64_t subs = (n + sub - 1) / sub;
    const uint64_t per = (subs + grid - 1) / grid;
    chunk = (per ? per : 1) * sub;
}

// Lanes of the wave holding the same digit as this lane (among `valid` lanes),
// found with one ballot per digit bit.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
        const uint32_t set = (d >> bit) & 1u;
        const uint64_t bb = __ballot(set != 0u);
        // lanes agreeing on this bit: bb where it is set, ~bb where it is not
        const uint32_t flip = set - 1u;
        m &= bb ^ (((uint64_t)flip << 32) | flip);
    }
    return m;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Per-wave LDS histograms.  match: lanes with equal digits are matched and the
// lowest of them adds the group's size (one LDS atomic per distinct digit per
// wave), for a pass whose digits are few (the depth keys' exponent byte), where
// per-key atomics on one address would serialise; otherwise one atomic per key.
// drop: keys equal to kCulledKey are left out (the compacting first pass of
// the depth order).
template <class K>
__global__ __launch_bounds__(kBlock) void k_hist(const K* __restrict__ keys, uint64_t n, int shift,
                                                 uint32_t dmask, uint64_t chunk, uint32_t grid,
                                                 bool drop, bool match,
                                                 uint32_t* __restrict__ hist,
                                                 const uint64_t* __restrict__ totals, int word,
                                                 uint32_t sub) {
    __shared__ uint32_t h[kWaves][kRadix];
    pass_extent(totals, word, sub, grid, n, chunk);
    for (int k = threadIdx.x; k < kWaves * kRadix; k += kBlock) (&h[0][0])[k] = 0u;
    __syncthreads();
    const uint64_t lo = (uint64_t)blockIdx.x * chunk;
    const uint64_t hi = lo + chunk < n ? lo + chunk : n;
    const int w = threadIdx.x >> 6;
    // kHistUnroll keys per lane and step, their loads issued together
    constexpr int kHistUnroll = 8;
    for (uint64_t base = lo; base < hi; base += kBlock * kHistUnroll) {   // uniform trip count
        K key[kHistUnroll];
#pragma unroll
        for (int u = 0; u < kHistUnroll; ++u) {
            const uint64_t i = base + (uint64_t)u * kBlock + threadIdx.x;
            key[u] = i < hi ? keys[i] : (K)0;
        }
#pragma unroll
        for (int u = 0; u < kHistUnroll; ++u) {
            const uint64_t i = base + (uint64_t)u * kBlock + threadIdx.x;
            const bool valid = i < hi && !(drop && key[u] == (K)kCulledKey);
            const uint32_t d = valid ? digit_of(key[u], shift, dmask) : 0u;
            if (match) {
                const uint64_t m = match_digit(d, valid);
                if (valid && lanes_below(m) == 0u) atomicAdd(&h[w][d], (uint32_t)__popcll(m));
            } else if (valid) {
                atomicAdd(&h[w][d], 1u);
            }
        }
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

// Exclusive scan of 256 values held one per lane of a 256-lane workgroup.
// `wsum` is 4 words of LDS.  Returns the exclusive prefix; *total gets the sum.
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t x, uint32_t* wsum,
                                                       uint32_t* total) {
    const uint32_t inc = wave_incl_scan32(x);
    const int w = threadIdx.x >> 6;
    if (__lane_id() == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
        before += k < w ? wsum[k] : 0u;
        all += wsum[k];
    }
    __syncthreads();
    *total = all;
    return before + inc - x;
}

// Workgroup d: exclusive scan over the grid counts of digit d, in place, and
// the digit total in hist[256 * grid + d].  grid <= 1024 = 256 lanes x 4.
__global__ __launch_bounds__(kBlock) void k_dscan(uint32_t* __restrict__ hist, uint32_t grid) {
    __shared__ uint32_t wsum[kWaves];
    uint32_t* row = hist + (uint64_t)blockIdx.x * grid;
    const uint32_t first = threadIdx.x * 4;
    uint32_t c[4], s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        c[k] = first + k < grid ? row[first + k] : 0u;
        s += c[k];
    }
    uint32_t total;
    uint32_t run = block_excl_scan256(s, wsum, &total);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (first + k < grid) row[first + k] = run;
        run += c[k];
    }
    if (threadIdx.x == 0) hist[(uint64_t)kRadix * grid + blockIdx.x] = total;
}

// vals_in == nullptr stands for the identity (value = input position);
// keys_out == nullptr skips the key writes (a last pass whose keys are unused);
// with gather_out, gather_out[p] = gather[value].w and sets_out[p] =
// gather[value] for every output position p (one 16-byte read per key);
// drop: keys equal to kCulledKey are left out, as in k_hist.  A workgroup
// walks its chunk in sub-tiles of kBlock * ITEMS keys.
template <class K, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_scatter(const K* __restrict__ keys_in,
                                                    const uint32_t* __restrict__ vals_in,
                                                    K* __restrict__ keys_out,
                                                    uint32_t* __restrict__ vals_out, uint64_t n,
                                                    int shift, uint32_t dmask, uint64_t chunk,
                                                    uint32_t grid, bool drop,
                                                    const uint32_t* __restrict__ hist,
                                                    const uint4* __restrict__ gather,
                                                    uint32_t* __restrict__ gather_out,
                                                    uint4* __restrict__ sets_out,
                                                    const uint64_t* __restrict__ totals,
                                                    int word) {
    constexpr int kItems = ITEMS;
    constexpr int kSub = kBlock * ITEMS;
    pass_extent(totals, word, (uint64_t)kSub, grid, n, chunk);
    __shared__ K s_key[kSub];
    __shared__ uint32_t s_val[kSub];
    __shared__ uint32_t base[kRadix];     // global position of this chunk's next key per digit
    __shared__ uint32_t lstart[kRadix];   // digit start within the current sub-tile
    __shared__ uint32_t tot[kRadix];      // digit count within the current sub-tile
    __shared__ uint32_t wcnt[kWaves][kRadix];
    __shared__ uint32_t wsum[kWaves];

    const int t = threadIdx.x;            // one digit per lane in the per-digit steps
    {
        uint32_t dummy;
        const uint32_t dstart =
            block_excl_scan256(hist[(uint64_t)kRadix * grid + t], wsum, &dummy);
        base[t] = dstart + hist[(uint64_t)t * grid + blockIdx.x];
    }
    const uint64_t lo = (uint64_t)blockIdx.x * chunk;
    const uint64_t hi = lo + chunk < n ? lo + chunk : n;
    const int w = t >> 6;
    const unsigned lane = __lane_id();
    for (uint64_t sub = lo; sub < hi; sub += kSub) {
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww) wcnt[ww][t] = 0u;
        __syncthreads();
        K key[kItems];
        uint32_t val[kItems];
        uint32_t rank[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const uint64_t idx = sub + (uint64_t)w * (64 * kItems) + (uint64_t)k * 64 + lane;
            const bool valid = idx < hi;
            key[k] = valid ? keys_in[idx] : (K)0;
            val[k] = valid ? (vals_in ? vals_in[idx] : (uint32_t)idx) : 0u;
        }
        // Rank = keys of the same digit in earlier items (the wave's running
        // count, advanced by each group's lowest lane with an LDS add that
        // returns the old count) + lanes below in the same group.  The adds
        // are issued back to back (a wave's LDS operations complete in order)
        // and their results read afterwards, so their latencies overlap.
        uint32_t pre[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const uint64_t idx = sub + (uint64_t)w * (64 * kItems) + (uint64_t)k * 64 + lane;
            const bool valid = idx < hi && !(drop && key[k] == (K)kCulledKey);
            const uint32_t d = digit_of(key[k], shift, dmask);
            const uint64_t m = match_digit(d, valid);
            const uint32_t below = lanes_below(m);
            pre[k] = 0u;
            if (valid && below == 0u) pre[k] = atomicAdd(&wcnt[w][d], (uint32_t)__popcll(m));
            // the group's lowest lane, and this lane's place in the group
            rank[k] = (m ? (uint32_t)__builtin_ctzll(m) : 0u) << 8 | below;
        }
#pragma unroll
        for (int k = 0; k < kItems; ++k)
            rank[k] = (uint32_t)__shfl((int)pre[k], (int)(rank[k] >> 8), 64) + (rank[k] & 255u);
        __syncthreads();
        {   // per digit: prefix over waves, sub-tile total, sub-tile digit start
            uint32_t s = 0;
#pragma unroll
            for (int ww = 0; ww < kWaves; ++ww) {
                const uint32_t c = wcnt[ww][t];
                wcnt[ww][t] = s;
                s += c;
            }
            tot[t] = s;
            uint32_t dummy;
            lstart[t] = block_excl_scan256(s, wsum, &dummy);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const uint64_t idx = sub + (uint64_t)w * (64 * kItems) + (uint64_t)k * 64 + lane;
            if (idx < hi && !(drop && key[k] == (K)kCulledKey)) {
                const uint32_t d = digit_of(key[k], shift, dmask);
                const uint32_t lp = lstart[d] + wcnt[w][d] + rank[k];
                if (lp < (uint32_t)kSub) {
                    s_key[lp] = key[k];
                    s_val[lp] = val[k];
                }
            }
        }
        __syncthreads();
        // keys kept in this sub-tile: the end of the last digit's run
        const uint32_t n_sub = lstart[kRadix - 1] + tot[kRadix - 1];
        // four staged keys per lane and step: their LDS reads overlap
        for (uint32_t i0 = t; i0 < n_sub; i0 += 4 * kBlock) {
            K kk[4];
            uint32_t v[4], pos[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t i = i0 + u * kBlock;
                const uint32_t ii = i < n_sub ? i : i0;
                kk[u] = s_key[ii];
                v[u] = s_val[ii];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t d = digit_of(kk[u], shift, dmask);
                pos[u] = base[d] + (i0 + u * kBlock - lstart[d]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (i0 + u * kBlock < n_sub && pos[u] < n) {
                    if (keys_out) keys_out[pos[u]] = kk[u];
                    vals_out[pos[u]] = v[u];
                    if (gather_out) {
                        const uint4 ts = gather[v[u]];
                        gather_out[pos[u]] = ts.w;
                        sets_out[pos[u]] = ts;
                    }
                }
            }
        }
        __syncthreads();
        base[t] += tot[t];
        __syncthreads();
    }
}

// One lane per boundary position i in [0, n]: every tile whose run starts at i
// gets start = i, every tile whose run ends at i gets end = i.
// Thread t covers the pair boundaries i = 4t .. 4t + 3 (i <= n): where the
// tile id changes between pair i - 1 and pair i (pair -1 counting as tile -1
// and pair n as tile n_tiles), the tiles in between end and start at i.
// Empty tiles get an empty range.
__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ keys, uint64_t n,
                                                int n_tiles, uint32_t* __restrict__ ranges,
                                                const uint64_t* __restrict__ totals) {
    n = frame_count(totals, 0, n);
    const uint64_t i0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4u;
    if (i0 > n) return;
    int k[5];
    k[0] = i0 == 0 ? -1 : (int)keys[i0 - 1];
    if (i0 + 4 <= n) {
        const uint4 v = *reinterpret_cast<const uint4*>(keys + i0);
        k[1] = (int)v.x; k[2] = (int)v.y; k[3] = (int)v.z; k[4] = (int)v.w;
    } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) k[1 + u] = i0 + u < n ? (int)keys[i0 + u] : n_tiles;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const uint64_t i = i0 + u;
        const int prev = k[u], cur = k[u + 1];
        if (i > n || prev == cur) continue;
        for (int t = prev + 1; t <= cur && t < n_tiles; ++t) ranges[2 * t] = (uint32_t)i;
        for (int t = prev < 0 ? 0 : prev; t < cur && t < n_tiles; ++t)
            ranges[2 * t + 1] = (uint32_t)i;
    }
}

// Sorts (key, value) pairs on the low `bits` key bits, ping-ponging between
// buffers 0 and 1 from buffer `cur`; *out_buf receives the buffer holding the
// result.  The first pass reads n0 pairs; with drop it leaves out the keys
// equal to kCulledKey, of which there must be n0 - n, and every later pass
// sorts the n kept pairs (without drop, n0 == n).  With `totals`, n is a
// bound and the passes that sort n keys read their count from device word
// `word` (and, without drop, so does the first).  identity: the input values
// are 0..n0-1 and are not read.  With last_keys false the final pass writes
// values only; with gather_out it also writes gather[value].w and (to
// sets_out) gather[value] in sorted order.
template <class K>
hipError_t radix_sort(K* keys[2], uint32_t* vals[2], int cur, uint64_t n0, uint64_t n, int bits,
                      uint32_t* tmp, bool drop, bool identity, bool last_keys,
                      const uint4* gather, uint32_t* gather_out, uint4* sets_out, int* out_buf,
                      hipStream_t s, const uint64_t* totals = nullptr, int word = 0) {
    // the bits are split as evenly as the passes allow, so no pass scatters
    // into more buckets than it must: the fewer the buckets, the longer each
    // sub-tile's runs of equal digits and its coalesced writes.  The wider
    // digits go to the last passes (13 bits: 6 + 7): the top bits of a tile
    // id take fewer values than their width allows (6500 tiles: 51 values of
    // bits 7-12, 102 of bits 6-12), the low bits all of theirs
    const int passes = (bits + 7) / 8;
    int shift = 0;
    for (int pass = 0; pass < passes; ++pass) {
        const uint64_t m = pass == 0 ? n0 : n;       // pairs this pass reads
        const Plan plan = make_plan(m);
        const int width = bits / passes + (pass >= passes - bits % passes ? 1 : 0);
        const uint32_t dmask = (1u << width) - 1u;
        const bool last = pass + 1 == passes;
        const bool dr = pass == 0 && drop;
        K* kout = (last && !last_keys) ? nullptr : keys[1 - cur];
        const uint32_t* vin = (pass == 0 && identity) ? nullptr : vals[cur];
        // the depth keys' top byte (sign and exponent) takes few values
        const bool match = drop && shift == 24;
        // the dropping first pass reads every slot, a host count
        const uint64_t* dc = (pass == 0 && drop) ? nullptr : totals;
        hipLaunchKernelGGL(k_hist<K>, dim3(plan.grid), dim3(kBlock), 0, s, keys[cur], m, shift,
                           dmask, plan.chunk, plan.grid, dr, match, tmp, dc, word,
                           (uint32_t)(kBlock * plan.items));
        hipLaunchKernelGGL(k_dscan, dim3(kRadix), dim3(kBlock), 0, s, tmp, plan.grid);
        auto scatter = plan.items == kItemsSmall ? k_scatter<K, kItemsSmall>
                                                 : k_scatter<K, kItemsLarge>;
        hipLaunchKernelGGL(scatter, dim3(plan.grid), dim3(kBlock), 0, s, keys[cur], vin, kout,
                           vals[1 - cur], m, shift, dmask, plan.chunk, plan.grid, dr, tmp, gather,
                           last ? gather_out : nullptr, last ? sets_out : nullptr, dc, word);
        cur = 1 - cur;
        shift += width;
    }
    *out_buf = cur;
    return hipGetLastError();
}

// Scratch of ss_sort_noalloc: one pass's per-workgroup digit counts and digit
// totals (kRadix x kMaxGrid + kRadix words, 1 MiB + 1 KiB, whatever the pair
// count), held on every GPU the library runs on until the process ends.  Every
// word a pass reads is written by that pass's k_hist and k_dscan first, so
// nothing needs clearing between calls; calls that overlap on one GPU share
// it and race.  In host code `scratch` names a host-side stand-in: kernels
// receive the device address hipGetSymbolAddress returns for the current
// device, looked up once per device.
constexpr int64_t kStaticSortWords = (int64_t)kRadix * kMaxGrid + kRadix;
static __device__ __align__(256) uint32_t scratch[kStaticSortWords];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch_ptr[kMaxDevices] = {};

hipError_t static_sort_scratch(uint32_t** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<uint32_t*>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

int sort_passes(int bits) { return (bits + 7) / 8; }

int64_t sort_tmp_words(uint64_t) { return (int64_t)kRadix * kMaxGrid + kRadix; }

int64_t static_sort_tmp_words() { return kStaticSortWords; }

hipError_t launch_depth_order(int64_t n, int64_t n_visible, const ss_frame& f, hipStream_t s,
                              const uint64_t* totals) {
    if (n <= 0 || n_visible <= 0) return hipSuccess;
    uint32_t* keys[2] = {f.depth_keys, f.depth_keys + n};
    uint32_t* vals[2] = {f.order, f.order + n};
    int out = 0;
    // 4 passes from buffer 0 end in buffer 0: the first drops the Gaussians
    // without tiles, the order lands in f.order[0, n_visible) and the last pass
    // writes the tile counts and the tile sets (to the start of emit_tmp) in
    // that order.
    return radix_sort<uint32_t>(keys, vals, 0, (uint64_t)n, (uint64_t)n_visible, 32, f.order_tmp,
                                true, true, false, reinterpret_cast<const uint4*>(f.tile_sets),
                                f.order_counts, reinterpret_cast<uint4*>(f.emit_tmp), &out, s,
                                totals, 1);
}

hipError_t launch_sort(const ss_pairs& p, int buf, uint64_t n, int bits, int* out_buf,
                       hipStream_t s, const uint64_t* totals) {
    uint32_t* keys[2] = {p.keys[0], p.keys[1]};
    uint32_t* vals[2] = {p.values[0], p.values[1]};
    if (n <= 1 && !totals) {
        *out_buf = buf;
        return hipSuccess;
    }
    if (n == 0) n = 1;      // a device count of 0 or 1 sorts nothing; the grid is one group
    return radix_sort<uint32_t>(keys, vals, buf, n, n, bits, p.sort_tmp, false, false, true,
                                nullptr, nullptr, nullptr, out_buf, s, totals, 0);
}

hipError_t launch_sort_static(const ss_pairs& p, int buf, uint64_t n, int bits, int* out_buf,
                              hipStream_t s) {
    if (sort_tmp_words(n) > kStaticSortWords) return hipErrorInvalidValue;
    ss_pairs q = p;
    const hipError_t e = static_sort_scratch(&q.sort_tmp);
    if (e != hipSuccess) return e;
    return launch_sort(q, buf, n, bits, out_buf, s);
}

hipError_t launch_ranges(const uint32_t* keys, uint64_t n, int n_tiles, uint32_t* ranges,
                         hipStream_t s, const uint64_t* totals) {
    const uint64_t threads = n / 4 + 1;           // boundaries 0 .. n, four per thread
    const uint64_t grid = (threads + 255) / 256;
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)grid), dim3(256), 0, s, keys, n, n_tiles, ranges,
                       totals);
    return hipGetLastError();
}

}  // namespace ss

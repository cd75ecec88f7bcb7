// Stage 3: key emission (Speedy-Splat Sec. 3.2.2, "duplicateWithKeys"; the
// "Process" step of Alg. 1).
//
// Entries are taken in depth order: entry j is Gaussian i = order[j], whose
// tiles go to [offsets[j] - counts[i], offsets[j]) as key = tile id, value = i.
// The emitted pairs are therefore sorted by (depth, index), and a stable sort
// on the tile id alone yields the paper's (tile | depth) order.  The order of
// one Gaussian's own pairs (distinct tiles) does not matter.
//
// Tile counts are heavy-tailed (most Gaussians touch a few tiles, a Gaussian
// near the camera thousands), so the work is split in two launches:
//   k_emit      one lane per entry whose tile set the preprocess stage stored
//               as a mask (tile rectangle within 8 x 8, so at most 64 tiles;
//               the depth order left the sets in entry order, so these reads
//               are coalesced); the wave deals its entries' pairs out to its
//               lanes (pair idx of the wave: owner by a binary search over
//               the wave's prefix of counts, tile by selecting the owner's
//               r-th mask bit), so consecutive lanes write consecutive
//               addresses and no lane walks a long mask while the others
//               wait.  Each workgroup lists its other entries
//               in its own segment of the scratch (no atomics: thousands on one
//               counter would serialise), and one workgroup turns the
//               per-segment counts into offsets;
//   k_emit_big  each wave takes 64 work items at a time, an item being a
//               run of a queued entry's bands (an entry of thousands of tiles
//               is split over up to 16 waves), and re-walks the FP64 tile
//               spans of their records: the spans (rows, or columns for
//               AccuTile on tall extents) of all 64 are dealt out to the
//               lanes, a wave prefix sum places them, and the wave writes the
//               keys with consecutive lanes on consecutive addresses.
#include "ss_internal.h"

namespace ss {
namespace {

constexpr int kBigBlock = 256;
constexpr int kBigGrid = 1024;
constexpr uint32_t kBigPartTiles = 512;   // tiles per part of a queued entry (at least)
constexpr int kBigParts = 16;             // parts of one queued entry at most

// Scratch layout for n entries, nb = ceil(n / 256) workgroups: segments of
// queued entries [0, 256 nb), their counts [256 nb, 257 nb), exclusive segment
// offsets with the total last [257 nb, 258 nb + 1), a coarse index
// [258 nb + 1, 262 nb + 2): word g names the segment holding queued entry
// 64 g, and per queued entry of more than one part a counter of the tiles
// its parts have placed [262 nb + 2, 518 nb + 2), at the entry's position in
// the queue.
__host__ __device__ __forceinline__ int64_t queue_blocks(int64_t n) { return (n + 255) / 256; }
__host__ __device__ __forceinline__ int64_t claim_offset(int64_t nb) { return 262 * nb + 2; }

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t x) {
    const int lane = (int)__lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// For two positions x0 <= x1 in a non-decreasing run of 64 LDS values s
// (s[0] <= x0): the last index whose value is <= x0, and the same for x1.
// Six steps of binary lifting each; the two searches are interleaved so that
// their LDS reads overlap.
__device__ __forceinline__ void last_le64x2(const uint32_t* s, uint32_t x0, uint32_t x1, int& a0,
                                            int& a1) {
    a0 = 0;
    a1 = 0;
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1) {
        const uint32_t v0 = s[a0 + step], v1 = s[a1 + step];
        a0 += v0 <= x0 ? step : 0;
        a1 += v1 <= x1 ? step : 0;
    }
}

// Orders the wave's LDS writes before its LDS reads by other lanes.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kEmitBlock = 256;
constexpr int kEmitWaves = kEmitBlock / 64;

// The bit index of the r-th (from 0) set bit of the 64-bit mask hi:lo, by
// halving: popcounts of the low half of the remaining window decide which
// half holds it.
__device__ __forceinline__ uint32_t select_bit64(uint32_t lo, uint32_t hi, uint32_t r) {
    const uint32_t pl = (uint32_t)__popc(lo);
    const bool up = r >= pl;
    uint32_t x = up ? hi : lo;
    uint32_t b = up ? 32u : 0u;
    r = up ? r - pl : r;
#pragma unroll
    for (uint32_t half = 16; half >= 1; half >>= 1) {
        const uint32_t c = (uint32_t)__popc(x & ((1u << half) - 1u));
        const bool u = r >= c;
        r = u ? r - c : r;
        x = u ? x >> half : x;
        b = u ? b + half : b;
    }
    return b;
}

__global__ __launch_bounds__(kEmitBlock) void k_emit(const Item* __restrict__ items,
                                                     BatchDims dims, uint32_t n_entries,
                                                     uint32_t limit,
                                                     const uint4* __restrict__ tsets,   // by entry
                                                     const uint32_t* __restrict__ order,
                                                     const uint32_t* __restrict__ offsets,
                                                     uint32_t* __restrict__ keys,
                                                     uint32_t* __restrict__ values,
                                                     uint32_t* __restrict__ queue,
                                                     const uint64_t* __restrict__ totals) {
    // n_entries (the queue layout) and limit are bounds; the counts of this
    // frame may be smaller (device frame counts)
    const uint32_t n_valid = (uint32_t)frame_count(totals, 1, n_entries);
    limit = (uint32_t)frame_count(totals, 0, limit);
    __shared__ uint32_t s_pre[kEmitWaves][64];    // exclusive prefix of the masked counts
    __shared__ uint32_t s_pos[kEmitWaves][64];    // first pair position of each lane's entry
    __shared__ uint32_t s_gid[kEmitWaves][64];
    __shared__ uint32_t s_mlo[kEmitWaves][64], s_mhi[kEmitWaves][64];   // the tile mask
    __shared__ uint32_t s_base[kEmitWaves][64];   // tile id of the mask window's bit 0
    __shared__ uint32_t s_txn[kEmitWaves][64];    // tiles per image row
    const int w = threadIdx.x >> 6;
    const int lane = (int)__lane_id();
    const int64_t j = (int64_t)blockIdx.x * kEmitBlock + threadIdx.x;   // depth-order entry
    const bool valid = j < n_valid;
    // offsets and order are independent loads, issued together
    const uint32_t end = valid ? offsets[j] : 0u;
    const uint32_t gid_j = valid ? order[j] : 0u;
    uint32_t prev = __shfl_up(end, 1, 64);
    if (lane == 0) prev = (valid && j > 0) ? offsets[j - 1] : 0u;
    const uint32_t cnt = valid ? end - prev : 0u;
    const uint32_t gid = cnt ? gid_j : 0u;
    uint4 ts = make_uint4(0u, 0u, 0u, 0u);
    if (cnt) ts = tsets[j];                       // the tile sets in depth order
    const uint64_t mask = (uint64_t)ts.x | ((uint64_t)ts.y << 32);
    const bool masked = cnt && mask != 0ull;
    const bool big = cnt && !masked;
    {   // list the big entries in this workgroup's segment
        __shared__ uint32_t s_nbig[kEmitWaves];
        const uint64_t bigs = __ballot(big);
        if (lane == 0) s_nbig[w] = (uint32_t)__popcll(bigs);
        __syncthreads();
        uint32_t before = 0, all = 0;
#pragma unroll
        for (int k = 0; k < kEmitWaves; ++k) {
            before += k < w ? s_nbig[k] : 0u;
            all += s_nbig[k];
        }
        const int64_t nb = queue_blocks(n_entries);
        if (big) {
            const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(bigs >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bigs, 0u));
            const int64_t slot = (int64_t)blockIdx.x * kEmitBlock + before + below;
            queue[slot] = (uint32_t)j;
            // the counter of an entry of more than one part starts at 0
            if (cnt > kBigPartTiles) queue[claim_offset(nb) + slot] = 0u;
        }
        if (threadIdx.x == 0) queue[nb * kEmitBlock + blockIdx.x] = all;
    }
    const uint32_t small = masked ? cnt : 0u;
    const uint32_t incl = wave_incl_scan_u32(small);
    const uint32_t total = __shfl(incl, 63, 64);
    if (total == 0u) return;                      // wave-uniform; no workgroup barrier follows
    s_pre[w][lane] = incl - small;
    s_pos[w][lane] = prev;
    s_gid[w][lane] = gid;
    s_mlo[w][lane] = ts.x;
    s_mhi[w][lane] = ts.y;
    if (small) {
        const Item& it = items[dims.n_items == 1 ? 0 : item_of_slot(items, dims.n_items, gid)];
        const uint32_t tx_n = (uint32_t)it.tx_n;
        s_base[w][lane] = (uint32_t)it.tile_off + (ts.z >> 16) * tx_n + (ts.z & 0xffffu);
        s_txn[w][lane] = tx_n;
    }
    wave_lds_sync();
    // the wave's pairs dealt out to its lanes: output idx belongs to the last
    // lane whose run starts at or before it, and is that lane's r-th tile
    for (uint32_t idx = (uint32_t)lane; idx < total; idx += 128) {
        const uint32_t idx2 = idx + 64;
        int a, a2;
        last_le64x2(s_pre[w], idx, idx2, a, a2);
        const uint32_t r = idx - s_pre[w][a];
        const uint32_t pos = s_pos[w][a] + r;
        if (pos < limit) {
            const uint32_t b = select_bit64(s_mlo[w][a], s_mhi[w][a], r);
            keys[pos] = s_base[w][a] + (b / kSetSide) * s_txn[w][a] + b % kSetSide;
            values[pos] = s_gid[w][a];
        }
        if (idx2 < total) {
            const uint32_t r2 = idx2 - s_pre[w][a2];
            const uint32_t pos2 = s_pos[w][a2] + r2;
            if (pos2 < limit) {
                const uint32_t b2 = select_bit64(s_mlo[w][a2], s_mhi[w][a2], r2);
                keys[pos2] = s_base[w][a2] + (b2 / kSetSide) * s_txn[w][a2] + b2 % kSetSide;
                values[pos2] = s_gid[w][a2];
            }
        }
    }
}

// One workgroup: exclusive offsets of the nb segment counts, total last, and
// the coarse index of every 64th queued entry.  Each lane scans kOffPer
// consecutive counts, so up to 4096 segments take one step.
constexpr int kOffPer = 4;
__global__ __launch_bounds__(1024) void k_emit_offsets(uint32_t* __restrict__ queue,
                                                       int64_t nb) {
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_carry;
    {
        uint32_t* base = queue;
        const uint32_t* cnt = base + nb * kEmitBlock;
        uint32_t* off = base + nb * kEmitBlock + nb;
        uint32_t* coarse = base + nb * kEmitBlock + 2 * nb + 1;
        if (threadIdx.x == 0) s_carry = 0u;
        __syncthreads();
        for (int64_t b = 0; b < nb; b += 1024 * kOffPer) {
            const int64_t b0 = b + (int64_t)threadIdx.x * kOffPer;
            uint32_t x[kOffPer], sum = 0;
#pragma unroll
            for (int k = 0; k < kOffPer; ++k) {
                x[k] = b0 + k < nb ? cnt[b0 + k] : 0u;
                sum += x[k];
            }
            const uint32_t inc = wave_incl_scan_u32(sum);
            const int w = threadIdx.x >> 6;
            if ((threadIdx.x & 63) == 63) s_w[w] = inc;
            __syncthreads();
            uint32_t before = s_carry;
            for (int k = 0; k < w; ++k) before += s_w[k];
            uint32_t o = before + inc - sum;
#pragma unroll
            for (int k = 0; k < kOffPer; ++k) {
                if (b0 + k < nb) {
                    off[b0 + k] = o;
                    for (uint32_t m = (o + 63u) & ~63u; m < o + x[k]; m += 64u)
                        coarse[m >> 6] = (uint32_t)(b0 + k);
                }
                o += x[k];
            }
            __syncthreads();
            if (threadIdx.x == 1023) s_carry = before + inc;
            __syncthreads();
        }
        if (threadIdx.x == 0) off[nb] = s_carry;
    }
}

// The depth-order entry at queue position q (< the total): the segment
// holding it is the last with offset <= q, between the segments holding
// positions 64 g and 64 (g + 1).  *at receives its index in the queue.
__device__ __forceinline__ uint32_t queue_entry(const uint32_t* __restrict__ base, int64_t nb,
                                                uint32_t q, uint32_t total, uint32_t* at) {
    const uint32_t* seg_off = base + nb * kEmitBlock + nb;
    const uint32_t* coarse = base + nb * kEmitBlock + 2 * nb + 1;
    const uint32_t g = q >> 6;
    int64_t lo = coarse[g];
    int64_t hi = (uint64_t)(g + 1) * 64u < total ? (int64_t)coarse[g + 1] : nb - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (seg_off[mid] <= q) lo = mid; else hi = mid - 1;
    }
    *at = (uint32_t)(lo * kEmitBlock + (q - seg_off[lo]));
    return base[*at];
}

__global__ __launch_bounds__(kBigBlock) void k_emit_big(const Item* __restrict__ items,
                                                        BatchDims dims, int mode, uint32_t limit,
                                                        int64_t nb,
                                                        const float4* __restrict__ geom,
                                                        const float4* __restrict__ conic,
                                                        const uint32_t* __restrict__ order,
                                                        const uint32_t* __restrict__ offsets,
                                                        uint32_t* __restrict__ keys,
                                                        uint32_t* __restrict__ values,
                                                        uint32_t* __restrict__ queue,
                                                        const uint64_t* __restrict__ totals) {
    constexpr int kW = kBigBlock / 64;
    // per band of the current chunk: start of its tiles in the chunk, tile id of
    // its first tile, tile id step along it, pair position of its first tile,
    // end of its entry's pair range, its Gaussian
    __shared__ uint32_t s_excl[kW][64];
    __shared__ uint32_t s_tile[kW][64];
    __shared__ uint32_t s_step[kW][64];
    __shared__ uint32_t s_pos[kW][64];
    __shared__ uint32_t s_end[kW][64];
    __shared__ uint32_t s_gid[kW][64];
    __shared__ uint32_t s_done[kW][64];      // tiles placed so far, per item of the round
    limit = (uint32_t)frame_count(totals, 0, limit);
    const int w = threadIdx.x >> 6;
    const int lane = (int)__lane_id();
    uint32_t* claim = queue + claim_offset(nb);
    const uint32_t nq = queue[nb * kEmitBlock + nb + nb];             // queued entries
    // Work item q is part q / nq_odd of queued entry q mod nq_odd (nq_odd: nq
    // rounded up to odd, so that one entry's parts land on different waves
    // whatever nq is).  An entry with c tiles over m bands has
    // p = min(ceil(c / kBigPartTiles), kBigParts) parts, part k taking bands
    // [k ceil(m / p), (k + 1) ceil(m / p)), so no wave walks all the bands of
    // a Gaussian that covers thousands of tiles; items past an entry's part
    // count do nothing.  Each round, lane l of the wave looks up item
    // wave0 + (64 r + l) waves, so that the chains of dependent loads
    // (segment search, entry, Gaussian, record) of 64 items overlap.  The
    // bands (tile rows, or columns for AccuTile on tall extents) of the
    // round's items are then dealt out to the lanes 64 at a time, each band's
    // span evaluated on its own as the preprocess stage counted it, and the
    // chunk's tiles written with consecutive lanes on consecutive pair
    // positions.  A band takes its place in its entry's pair range with an
    // add that returns the tiles placed before it (in LDS for an entry of one
    // part, else on the entry's counter in the scratch, which k_emit zeroed):
    // the order of one Gaussian's own pairs does not matter.
    const uint32_t nq_odd = nq | 1u;
    const uint64_t n_items = nq ? (uint64_t)nq_odd * kBigParts : 0u;
    const uint32_t wave0 = blockIdx.x * kW + w;
    const uint32_t waves = gridDim.x * kW;
    for (uint32_t r0 = 0; wave0 + (uint64_t)r0 * waves < n_items; r0 += 64) {
        const uint64_t iq = wave0 + (uint64_t)(r0 + lane) * waves;
        const uint32_t b = iq < n_items ? (uint32_t)(iq % nq_odd) : nq;
        const uint32_t part = iq < n_items ? (uint32_t)(iq / nq_odd) : 0u;
        Ellipse e;
        e.u = e.v = e.a = e.b = e.c = e.t = e.det = e.hx = e.hy = 0.0;
        e.x0 = e.x1 = e.y0 = e.y1 = 0;
        e.cols = false;
        bool ok = false;
        uint32_t i = 0, pos0 = 0, end = 0, tile_off = 0, np = 0, slot = 0, j = 0;
        int tx_n = 0, ty_n = 0, by0 = 0, by1 = 0;
        const bool have = b < nq;
        if (have) j = queue_entry(queue, nb, b, nq, &slot);           // depth-order entry
        if (have) {
            pos0 = j > 0 ? offsets[j - 1] : 0u;
            end = offsets[j];
            const uint32_t np0 = (end - pos0 + kBigPartTiles - 1) / kBigPartTiles;
            np = np0 < (uint32_t)kBigParts ? np0 : (uint32_t)kBigParts;
            if (part < np) {
                i = order[j];
                const Item& it =
                    items[dims.n_items == 1 ? 0 : item_of_slot(items, dims.n_items, i)];
                tx_n = it.tx_n;
                ty_n = it.ty_n;
                by0 = it.by0;
                by1 = it.by1;
                tile_off = (uint32_t)it.tile_off;
                ok = ellipse_setup(geom[kRec * (uint64_t)i], conic[kRec * (uint64_t)i], mode,
                                   tx_n, ty_n, by0, by1, e);
            }
        }
        const bool cols = ok && span_columns(e, mode);
        const uint32_t m_all =
            ok ? (uint32_t)(cols ? e.x1 - e.x0 + 1 : e.y1 - e.y0 + 1) : 0u;
        // this item's bands [kb0, kb0 + nmaj) of the entry's m_all
        const uint32_t per = np ? (m_all + np - 1) / np : 0u;
        const uint32_t kb0 = part * per < m_all ? part * per : m_all;
        const uint32_t kb1 = kb0 + per < m_all ? kb0 + per : m_all;
        const uint32_t nmaj = kb1 - kb0;
        const uint32_t incl = wave_incl_scan_u32(nmaj);
        const uint32_t n_bands = __shfl(incl, 63, 64);
        s_done[w][lane] = 0u;
        wave_lds_sync();
        for (uint32_t c0 = 0; c0 < n_bands; c0 += 64) {
            const uint32_t jb = c0 + (uint32_t)lane;
            // owner L: the first lane whose inclusive band count exceeds jb
            int L = 0;
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1) {
                const uint32_t v = (uint32_t)__shfl((int)incl, L + step - 1, 64);
                if (v <= jb) L += step;
            }
            L = L > 63 ? 63 : L;
            const int k = (int)(jb - ((uint32_t)__shfl((int)incl, L, 64) -
                                      (uint32_t)__shfl((int)nmaj, L, 64))) +
                          __shfl((int)kb0, L, 64);
            Ellipse el;
            el.u = __shfl(e.u, L, 64); el.v = __shfl(e.v, L, 64);
            el.a = __shfl(e.a, L, 64); el.b = __shfl(e.b, L, 64); el.c = __shfl(e.c, L, 64);
            el.t = __shfl(e.t, L, 64); el.det = __shfl(e.det, L, 64);
            el.hx = __shfl(e.hx, L, 64); el.hy = __shfl(e.hy, L, 64);
            el.x0 = __shfl(e.x0, L, 64); el.x1 = __shfl(e.x1, L, 64);
            el.y0 = __shfl(e.y0, L, 64); el.y1 = __shfl(e.y1, L, 64);
            const bool cl = __shfl((int)cols, L, 64) != 0;
            el.cols = cl;
            const int row0 = __shfl(by0, L, 64);    // the item's first tile row
            const int txn = __shfl(tx_n, L, 64), tyn = __shfl(ty_n, L, 64);
            const uint32_t gi = __shfl(i, L, 64), p0 = __shfl(pos0, L, 64);
            const uint32_t pend = __shfl(end, L, 64), toff = __shfl(tile_off, L, 64);
            const uint32_t pnp = __shfl(np, L, 64), pslot = __shfl(slot, L, 64);
            int lo = 0, hi = -1;
            if (jb < n_bands) {
                if (mode == SS_TILE_ACCUTILE) {
                    accutile_band(el, cl, k, txn, tyn, lo, hi);
                } else {
                    lo = el.x0;
                    hi = el.x1;
                }
            }
            const uint32_t len = hi >= lo ? (uint32_t)(hi - lo + 1) : 0u;
            uint32_t start = 0u;
            if (len) start = pnp > 1u ? atomicAdd(claim + pslot, len) : atomicAdd(&s_done[w][L], len);
            const int major = (cl ? el.x0 : el.y0) + k;
            // tile id of the band's minor index m: rows toff + (major - row0) txn + m,
            // columns toff + (m - row0) txn + major
            const uint32_t t_lo = cl ? toff + (uint32_t)((lo - row0) * txn + major)
                                     : toff + (uint32_t)((major - row0) * txn + lo);
            const uint32_t cincl = wave_incl_scan_u32(len);
            const uint32_t ctotal = __shfl(cincl, 63, 64);
            s_excl[w][lane] = cincl - len;
            s_tile[w][lane] = t_lo;
            s_step[w][lane] = cl ? (uint32_t)txn : 1u;
            s_pos[w][lane] = p0 + start;
            s_end[w][lane] = pend;
            s_gid[w][lane] = gi;
            wave_lds_sync();
            for (uint32_t idx = lane; idx < ctotal; idx += 128) {
                // the last bands whose exclusive starts are <= idx, idx + 64
                int ab[2];
                last_le64x2(s_excl[w], idx, idx + 64, ab[0], ab[1]);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const uint32_t ix = idx + 64u * h;
                    const int a = ab[h];
                    const uint32_t off = ix - s_excl[w][a];
                    const uint32_t pos = s_pos[w][a] + off;
                    if (ix < ctotal && pos < s_end[w][a] && pos < limit) {
                        keys[pos] = s_tile[w][a] + off * s_step[w][a];
                        values[pos] = s_gid[w][a];
                    }
                }
            }
            wave_lds_sync();
        }
    }
}

}  // namespace

int64_t emit_tmp_words(int64_t n) {
    const int64_t nb = queue_blocks(n);
    // the depth-ordered tile sets (4 words per entry), then the queue
    const int64_t q = 4 * n + claim_offset(nb) + nb * kEmitBlock;
    const int64_t pre = 2 * ((n + 63) / 64);     // the preprocess stage's partial counts
    return q > pre ? q : pre;
}

hipError_t launch_emit(const Item* items, const BatchDims& d, int mode, const ss_frame& f,
                       int64_t n_entries, uint32_t* keys, uint32_t* values, uint64_t n_pairs,
                       hipStream_t s, const uint64_t* totals) {
    if (n_entries <= 0) return hipSuccess;
    const int64_t nb = queue_blocks(n_entries);
    // emit_tmp: the depth-ordered tile sets the depth order left, then the queue
    const uint4* sets = reinterpret_cast<const uint4*>(f.emit_tmp);
    uint32_t* queue = f.emit_tmp + 4 * n_entries;
    hipLaunchKernelGGL(k_emit, dim3((unsigned)nb), dim3(kEmitBlock), 0, s, items, d,
                       (uint32_t)n_entries, (uint32_t)n_pairs, sets, f.order, f.offsets, keys,
                       values, queue, totals);
    hipLaunchKernelGGL(k_emit_offsets, dim3(1), dim3(1024), 0, s, queue, nb);
    hipLaunchKernelGGL(k_emit_big, dim3(kBigGrid), dim3(kBigBlock), 0, s, items, d, mode,
                       (uint32_t)n_pairs, nb, reinterpret_cast<const float4*>(f.geom),
                       reinterpret_cast<const float4*>(f.conic), f.order, f.offsets, keys,
                       values, queue, totals);
    return hipGetLastError();
}

}  // namespace ss

// Stage 6: per-tile front-to-back alpha blending (Speedy-Splat Sec. 3.2.3,
// Eqs. render_alpha, 2d_gaussian_scalar and contribution).
//
// One wave (64 lanes) per 16x16 tile.  Lane l owns column l % 16 and rows
// l / 16 + 4s of the four 16x4 strips s = 0..3, so the dx-dependent terms of
// q are computed once per lane and Gaussian and shared by its four pixels, and
// a strip's included-pixel work is skipped as a unit when none of its 64
// pixels lies inside the ellipse.  The tile's sorted Gaussians are staged
// through LDS 64 at a time (one gathered record per lane); the next batch's
// records are loaded into registers while the current batch is blended.
//
// A pixel that has finished (the next Gaussian would take its transmittance
// below 1e-4) moves its sample row to y = 1e30, so its q <= t test fails from
// then on; every 8 Gaussians a ballot per strip marks strips whose 64 pixels
// have all finished, which then skip their work, and the wave stops once
// every pixel has finished.  The quadratic form is evaluated with two fused
// multiply-adds as q = fma(dy, fma(c, dy, (2b) dx), (a dx) dx) and compared
// with the record's t, so the inclusion test (alpha >= 1/255) is exact and
// reproducible.  An included strip takes a short path when none of its
// pixels stops at this Gaussian (wave-uniform test) and the full path, which
// freezes the stopping pixels, otherwise.  Nothing on this path is a dense
// contraction, so it runs on the FP32 VALU.
#include "ss_internal.h"

namespace ss {
namespace {

constexpr int kBatch = 64;
constexpr float kDone = 1e30f;                    // sample row of a finished pixel
constexpr float kNegHalfLog2e = -0.72134752044448170368f;  // -log2(e) / 2

struct Rec {
    float4 g;   // (u, v, -, t)
    float4 q;   // (a, 2b, c, sigma)
    float4 c;   // (r, g, b, -)
};

__device__ __forceinline__ Rec make_rec0() {
    Rec r;
    r.g = r.q = r.c = make_float4(0.f, 0.f, 0.f, 0.f);
    return r;
}

// The record of list entry min(j, last): loads with no condition, so the
// compiler keeps them in flight until the values are used.
__device__ __forceinline__ uint32_t entry_gid(const uint32_t* __restrict__ values, uint32_t j,
                                              uint32_t last) {
    return values[j < last ? j : last];
}

__device__ __forceinline__ Rec load_rec(const float4* __restrict__ geom,
                                        const float4* __restrict__ conic,
                                        const float4* __restrict__ rgb, uint32_t gi) {
    Rec r;
    r.g = geom[gi];
    r.q = conic[gi];
    r.c = rgb[gi];
    return r;
}

// Tile work order: the tiles by decreasing list length (in buckets of 8
// entries; tiles within a bucket in no particular order).  Workgroups are
// dispatched in launch order, so the longest tiles start first and the short
// ones fill the gaps they leave, instead of a long tile that starts late
// running on alone at the end of the launch.  One workgroup.
constexpr int kOrderBuckets = 1024;

__device__ __forceinline__ uint32_t order_bucket(uint32_t len) {
    const uint32_t b = len >> 3;
    return b < (uint32_t)kOrderBuckets - 1u ? b : (uint32_t)kOrderBuckets - 1u;
}

__global__ __launch_bounds__(1024) void k_tile_order(const uint32_t* __restrict__ ranges,
                                                     int n_tiles, uint32_t* __restrict__ order) {
    __shared__ uint32_t h[kOrderBuckets];
    __shared__ uint32_t s_w[1024 / 64];
    const int t0 = (int)threadIdx.x;
    h[t0] = 0u;
    __syncthreads();
    for (int t = t0; t < n_tiles; t += 1024)
        atomicAdd(&h[order_bucket(ranges[2 * t + 1] - ranges[2 * t])], 1u);
    __syncthreads();
    // start of bucket b: the number of tiles in buckets above b
    const uint32_t x = h[kOrderBuckets - 1 - t0];
    uint32_t incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(incl, d, 64);
        if ((t0 & 63) >= d) incl += y;
    }
    if ((t0 & 63) == 63) s_w[t0 >> 6] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (int k = 0; k < (t0 >> 6); ++k) before += s_w[k];
    h[kOrderBuckets - 1 - t0] = before + incl - x;
    __syncthreads();
    for (int t = t0; t < n_tiles; t += 1024) {
        const uint32_t pos = atomicAdd(&h[order_bucket(ranges[2 * t + 1] - ranges[2 * t])], 1u);
        order[pos] = (uint32_t)t;
    }
}

template <bool STATS>
__global__ __launch_bounds__(64) void k_blend(const Item* __restrict__ items, BatchDims dims,
                                              const uint32_t* __restrict__ tile_order,
                                              const uint32_t* __restrict__ ranges,
                                              const uint32_t* __restrict__ values,
                                              const float4* __restrict__ geom,
                                              const float4* __restrict__ conic,
                                              const float4* __restrict__ rgb,
                                              float* __restrict__ out_single,
                                              float* __restrict__ t_final_all,
                                              uint32_t* __restrict__ n_last_all,
                                              uint32_t* __restrict__ n_eval_all,
                                              uint32_t* __restrict__ n_contrib_all) {
    __shared__ float4 s_geo[kBatch];
    __shared__ float4 s_con[kBatch];
    __shared__ float4 s_col[kBatch];
    if ((int)blockIdx.x >= dims.n_tiles) return;
    const int tile = (int)tile_order[blockIdx.x];
    const Item& it = items[dims.n_items == 1 ? 0 : item_of_tile(items, dims.n_items, tile)];
    const int W = it.cam.width, H = it.cam.height, tx_n = it.tx_n;
    const float bg0 = it.cam.bg[0], bg1 = it.cam.bg[1], bg2 = it.cam.bg[2];
    float* __restrict__ out = out_single ? out_single : it.out_rgb;
    float* __restrict__ t_final = t_final_all + it.pix_off;
    uint32_t* __restrict__ n_last = n_last_all + it.pix_off;
    uint32_t* __restrict__ n_eval = STATS ? n_eval_all + it.pix_off : nullptr;
    uint32_t* __restrict__ n_contrib =
        STATS && n_contrib_all ? n_contrib_all + it.pix_off : nullptr;
    const int lt = tile - it.tile_off;      // tile within the item's image
    const int lane = (int)threadIdx.x;
    const int tx = lt % tx_n, ty = lt / tx_n;
    const int px = tx * kTile + (lane & 15);
    const int py0 = ty * kTile + (lane >> 4);
    const float fx = (float)px + 0.5f;
    float fy[4], T[4], C[4][3];
    uint32_t last[4], stop[4], ncon[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const bool in = px < W && (py0 + 4 * s) < H;
        fy[s] = in ? (float)(py0 + 4 * s) + 0.5f : kDone;
        T[s] = 1.0f;
        C[s][0] = C[s][1] = C[s][2] = 0.0f;
        last[s] = 0u;
        stop[s] = 0u;
        ncon[s] = 0u;
    }
    uint32_t sl = 0;                              // bit s: strip s has an unfinished pixel
#pragma unroll
    for (int s = 0; s < 4; ++s) sl |= (__ballot(fy[s] < kDone) != 0ull ? 1u : 0u) << s;
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
    // Batch b's records are fetched during batch b - 1 and their list entries
    // during batch b - 2, so neither load stalls a batch.  Entries past the
    // list end repeat its last entry (in bounds, never read from LDS).
    const uint32_t e_last = end > start ? end - 1 : start;
    Rec nxt = make_rec0();
    uint32_t gid_nx = 0;
    if (start < end) {
        nxt = load_rec(geom, conic, rgb, entry_gid(values, start + lane, e_last));
        gid_nx = entry_gid(values, start + kBatch + lane, e_last);
    }
    for (uint32_t base = start; base < end && sl; base += kBatch) {
        s_geo[lane] = nxt.g;
        s_con[lane] = make_float4(nxt.q.x, 2.0f * nxt.q.y, nxt.q.z, nxt.q.w);
        s_col[lane] = nxt.c;
        __syncthreads();
        nxt = load_rec(geom, conic, rgb, gid_nx);
        gid_nx = entry_gid(values, base + 2 * kBatch + lane, e_last);
        const uint32_t nb = end - base < (uint32_t)kBatch ? end - base : (uint32_t)kBatch;

        for (uint32_t k = 0; k < nb; ++k) {
            const float4 g = s_geo[k];
            const float4 q = s_con[k];
            const float4 c = s_col[k];
            const float dx = fx - g.x;
            const float adx2 = (q.x * dx) * dx;
            const float b2dx = q.y * dx;
            const uint32_t pos = base + k - start + 1u;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                if (!(sl & (1u << s))) continue;      // wave-uniform
                const float dy = fy[s] - g.y;
                const float qq = fmaf(dy, fmaf(q.z, dy, b2dx), adx2);
                if (qq <= g.w) {
                    const float al = fminf(kAlphaMax, q.w * __builtin_amdgcn_exp2f(qq * kNegHalfLog2e));
                    float tn = T[s] * (1.0f - al);
                    float wgt = al * T[s];
                    uint32_t lp = pos;
                    uint32_t blended = 1u;
                    if (__ballot(tn < kTMin) != 0ull) {   // some included pixel stops here
                        const bool ok = tn >= kTMin;
                        wgt = ok ? wgt : 0.0f;
                        tn = ok ? tn : T[s];
                        lp = ok ? pos : last[s];
                        fy[s] = ok ? fy[s] : kDone;
                        if (STATS) stop[s] = ok ? stop[s] : pos;
                        blended = ok ? 1u : 0u;
                    }
                    if (STATS) ncon[s] += blended;
                    C[s][0] = fmaf(c.x, wgt, C[s][0]);
                    C[s][1] = fmaf(c.y, wgt, C[s][1]);
                    C[s][2] = fmaf(c.z, wgt, C[s][2]);
                    T[s] = tn;
                    last[s] = lp;
                }
            }
            if ((k & 7u) == 7u) {
                uint32_t now = 0;
#pragma unroll
                for (int s = 0; s < 4; ++s) now |= (__ballot(fy[s] < kDone) != 0ull ? 1u : 0u) << s;
                sl &= now;
                if (!sl) break;
            }
        }
        __syncthreads();
    }
    const size_t hw = (size_t)W * (size_t)H;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int py = py0 + 4 * s;
        if (px < W && py < H) {
            const size_t p = (size_t)py * W + px;
            out[p] = C[s][0] + T[s] * bg0;
            out[hw + p] = C[s][1] + T[s] * bg1;
            out[2 * hw + p] = C[s][2] + T[s] * bg2;
            t_final[p] = T[s];
            n_last[p] = last[s];
            if (STATS) n_eval[p] = stop[s] ? stop[s] : end - start;
            if (STATS && n_contrib) n_contrib[p] = ncon[s];
        }
    }
}

}  // namespace

hipError_t launch_blend(const Item* items, const BatchDims& d, const ss_frame& f,
                        const uint32_t* values, float* out_rgb_single, hipStream_t s) {
    const int grid = d.n_tiles;
    if (grid == 0) return hipSuccess;
    uint32_t* order = tile_order_of(f.table, d.n_items);
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(1024), 0, s, f.ranges, d.n_tiles, order);
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(64), 0, s, items, d, order, f.ranges, values,
                           reinterpret_cast<const float4*>(f.geom),
                           reinterpret_cast<const float4*>(f.conic),
                           reinterpret_cast<const float4*>(f.rgb), out_rgb_single, f.t_final,
                           f.n_last, f.n_eval, f.n_contrib);
    };
    if (f.n_eval) go(k_blend<true>);
    else go(k_blend<false>);
    return hipGetLastError();
}

}  // namespace ss

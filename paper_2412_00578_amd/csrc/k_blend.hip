// Stage 6: per-tile front-to-back alpha blending (Speedy-Splat Sec. 3.2.3,
// Eqs. render_alpha, 2d_gaussian_scalar and contribution).
//
// One wave (64 lanes) per 16x16 tile.  Lane l owns column l % 16 and rows
// l / 16 + 4s of the four 16x4 strips s = 0..3, so the dx-dependent terms of
// q are computed once per lane and Gaussian and shared by its four pixels, and
// a strip's included-pixel work is skipped as a unit when none of its 64
// pixels lies inside the ellipse.  The tile's sorted Gaussians are staged
// through LDS 64 at a time (one gathered record per lane); the next batch's
// records are loaded into registers while the current batch is blended.  A
// batch is walked in fully unrolled groups of 8 entries, the last group padded
// with records that include no pixel, so loop control is paid once per group.
//
// A pixel that has finished (the next Gaussian would take its transmittance
// below 1e-4) moves its sample row to y = 1e30, so its q <= t test fails from
// then on, and after every group a ballot stops the wave once every pixel has
// finished.  Strips are not tested for liveness one by one: the scalar test
// and branch per strip and Gaussian cost more issue slots than the four
// vector operations a finished strip's failing q <= t test takes.  The
// quadratic form of the stored record is evaluated in FP64, with dx and dy
// from one subtraction each and q = fma(fma(c, dy, (2b) dx), dy, (a dx) dx),
// and compared with the record's t: the inclusion test (alpha >= 1/255) is
// the inequality the tile geometry decides in FP64 on the same record, so a
// pixel is included only where its tile was assigned, and an ill-conditioned
// q (a needle-like Gaussian seen along its long axis) keeps its accuracy.
// The four strips' q are evaluated before any of their inclusion branches, so
// their FP64 dependency chains overlap instead of each waiting behind the
// previous strip's branch.  FP64
// adds and FMAs issue at the rate of FP32 ones, and the record is staged in
// LDS already widened.  alpha = sigma exp(-q/2) is evaluated in FP32 as
// exp2(fma(q, -log2(e)/2, log2 sigma)) with log2 sigma taken once per staged
// record: one multiply fewer per included strip, within the few-ulp error any
// faithful exp has.  An included
// strip takes a short path when none of its pixels stops at this Gaussian
// (wave-uniform test) and the full path, which freezes the stopping pixels,
// otherwise.  Nothing on this path is a dense contraction, so it runs on the
// FP32 VALU.
#include "ss_internal.h"

namespace ss {
namespace {

constexpr int kBatch = 64;
constexpr double kDone = 1e30;                    // sample row of a finished pixel
constexpr float kNegHalfLog2e = -0.72134752044448170368f;  // -log2(e) / 2

struct Rec {
    float4 g;   // (u, v, -, t)
    float4 q;   // (a, 2b, c, sigma); staged in LDS as (a, 2b, c, log2 sigma)
    float4 c;   // (r, g, b, -)
};

__device__ __forceinline__ bool unfinished(const double (&fy)[4]) {
    return fy[0] < kDone || fy[1] < kDone || fy[2] < kDone || fy[3] < kDone;
}

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
    r.g = geom[kRec * (uint64_t)gi];
    r.q = conic[kRec * (uint64_t)gi];
    r.c = rgb[gi];
    return r;
}

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) d2v lds_d2v;
typedef __attribute__((address_space(3))) f4v lds_f4v;

// The records of a tile's list staged in LDS, kBatch at a time.
struct Stage {
    double2 uv[kBatch];     // (u, v)
    double2 ab[kBatch];     // (a, 2b)
    double2 ct[kBatch];     // (c, t)
    float4 col[kBatch];     // (r, g, b, log2 sigma)
};

template <bool STATS>
__device__ __forceinline__ void blend_tile(const int tile, Stage& st,
                                           const Item* __restrict__ items, const BatchDims& dims,
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
    double2* __restrict__ s_uv = st.uv;
    double2* __restrict__ s_ab = st.ab;
    double2* __restrict__ s_ct = st.ct;
    float4* __restrict__ s_col = st.col;
    const Item& it = items[dims.n_items == 1 ? 0 : item_of_tile(items, dims.n_items, tile)];
    const int W = it.cam.width, H = it.cam.height, tx_n = it.tx_n;
    const float bg0 = it.cam.bg[0], bg1 = it.cam.bg[1], bg2 = it.cam.bg[2];
    float* __restrict__ out = out_single ? out_single : it.out_rgb;
    float* __restrict__ t_final = t_final_all + it.pix_off;
    uint32_t* __restrict__ n_last = n_last_all + it.pix_off;
    uint32_t* __restrict__ n_eval = STATS ? n_eval_all + it.pix_off : nullptr;
    uint32_t* __restrict__ n_contrib =
        STATS && n_contrib_all ? n_contrib_all + it.pix_off : nullptr;
    const int lt = tile - it.tile_off;      // tile within the item's band of tile rows
    const int lane = (int)threadIdx.x;
    const int tx = lt % tx_n, ty = lt / tx_n + it.by0;
    const int row0 = it.by0 * kTile;        // first image row of the band
    const int px = tx * kTile + (lane & 15);
    const int py0 = ty * kTile + (lane >> 4);
    const double fx = (double)px + 0.5;
    double fy[4];
    float T[4], C[4][3];
    uint32_t last[4], stop[4], ncon[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const bool in = px < W && (py0 + 4 * s) < H;
        fy[s] = in ? (double)(py0 + 4 * s) + 0.5 : kDone;
        T[s] = 1.0f;
        C[s][0] = C[s][1] = C[s][2] = 0.0f;
        last[s] = 0u;
        stop[s] = 0u;
        ncon[s] = 0u;
    }
    bool live = __ballot(unfinished(fy)) != 0ull;  // some pixel of the tile is unfinished
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
    for (uint32_t base = start; base < end && live; base += kBatch) {
        // slots past the list end hold a record whose q is 0 at every pixel
        // and whose t is -1, so it includes no pixel
        const bool real = base + (uint32_t)lane < end;
        s_uv[lane] = real ? make_double2(nxt.g.x, nxt.g.y) : make_double2(0.0, 0.0);
        s_ab[lane] = real ? make_double2(nxt.q.x, 2.0 * (double)nxt.q.y) : make_double2(0.0, 0.0);
        s_ct[lane] = real ? make_double2(nxt.q.z, nxt.g.w) : make_double2(0.0, -1.0);
        s_col[lane] = make_float4(nxt.c.x, nxt.c.y, nxt.c.z,
                                  real ? __builtin_amdgcn_logf(nxt.q.w) : 0.0f);
        __syncthreads();
        nxt = load_rec(geom, conic, rgb, gid_nx);
        gid_nx = entry_gid(values, base + 2 * kBatch + lane, e_last);
        const uint32_t nb = end - base < (uint32_t)kBatch ? end - base : (uint32_t)kBatch;

        // groups of 8 entries, the last one padded; the tile stops once every
        // pixel has finished
        const uint32_t nb8 = (nb + 7u) & ~7u;
        for (uint32_t k0 = 0; k0 < nb8; k0 += 8u) {
            // the group's first staged record as one LDS address held in a
            // vector register for its eight entries (each entry's four
            // reads take it with an immediate offset)
            uint32_t ga = (uint32_t)(uintptr_t)(const lds_d2v*)(s_uv + k0);
            asm volatile("" : "+v"(ga));
            const lds_d2v* __restrict__ g2 = (const lds_d2v*)(uintptr_t)ga;
            const lds_f4v* __restrict__ g4 = (const lds_f4v*)(uintptr_t)ga;
#pragma unroll
            for (uint32_t u = 0; u < 8u; ++u) {
                const uint32_t k = k0 + u;
                const d2v uv = g2[u];
                const d2v ab = g2[kBatch + u];
                const d2v ct = g2[2 * kBatch + u];
                const f4v c = g4[3 * kBatch + u];
                const double dx = fx - uv.x;
                const double adx2 = (ab.x * dx) * dx;
                const double b2dx = ab.y * dx;
                const uint32_t pos = base + k - start + 1u;
                // the four strips' FP64 chains first, so their latencies overlap
                double q4[4];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const double dy = fy[s] - uv.y;
                    q4[s] = fma(fma(ct.x, dy, b2dx), dy, adx2);
                }
                // keeps the compiler from sinking each chain into its branch
                asm volatile("" : "+v"(q4[0]), "+v"(q4[1]), "+v"(q4[2]), "+v"(q4[3]));
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const double qq = q4[s];
                    if (qq <= ct.y) {
                        const float al = fminf(kAlphaMax, __builtin_amdgcn_exp2f(
                                                              fmaf((float)qq, kNegHalfLog2e, c.w)));
                        float tn = T[s] * (1.0f - al);
                        float wgt = al * T[s];
                        uint32_t lp = pos;
                        uint32_t blended = 1u;
                        // rare: an included pixel stops here
                        if (__builtin_expect(__ballot(tn < kTMin) != 0ull, 0)) {
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
            }
            live = __ballot(unfinished(fy)) != 0ull;
            if (!live) break;
        }
        __syncthreads();
    }
    const int rows = (H < it.by1 * kTile ? H : it.by1 * kTile) - row0;   // the band's rows
    const size_t hw = (size_t)W * (size_t)rows;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int py = py0 + 4 * s;
        if (px < W && py < H) {
            const size_t p = (size_t)(py - row0) * W + px;
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

// One workgroup (one wave) per tile, tiles taken in the work order: launch
// index b renders tile tile_order[b].
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
    __shared__ Stage st;
    if ((int)blockIdx.x >= dims.n_tiles) return;
    blend_tile<STATS>((int)tile_order[blockIdx.x], st, items, dims, ranges, values, geom, conic,
                      rgb, out_single, t_final_all, n_last_all, n_eval_all, n_contrib_all);
}

// Persistent: a grid the GPU holds at once (a multiple of 8 workgroups) pulls
// tiles from per-XCD work queues until they are empty.  Workgroup b runs on
// XCD b mod 8 and takes the tiles the work order gave that XCD (launch indices
// x + 8 r, longest lists first) by incrementing the XCD's counter (zeroed by
// k_tile_order); no workgroup waits on another.  Serves a batch's tiles of
// every item and resolution from one resident grid.
template <bool STATS>
__global__ __launch_bounds__(64) void k_blend_persistent(
    const Item* __restrict__ items, BatchDims dims, const uint32_t* __restrict__ tile_order,
    uint32_t* __restrict__ queue, const uint32_t* __restrict__ ranges,
    const uint32_t* __restrict__ values, const float4* __restrict__ geom,
    const float4* __restrict__ conic, const float4* __restrict__ rgb,
    float* __restrict__ out_single, float* __restrict__ t_final_all,
    uint32_t* __restrict__ n_last_all, uint32_t* __restrict__ n_eval_all,
    uint32_t* __restrict__ n_contrib_all) {
    __shared__ Stage st;
    const uint32_t x = blockIdx.x & 7u;
    const uint32_t n = (uint32_t)dims.n_tiles;
    const uint32_t cap = n > x ? (n - x + 7u) / 8u : 0u;    // launch indices of XCD x
    for (;;) {
        uint32_t r = 0u;
        if (threadIdx.x == 0) r = atomicAdd(queue + x, 1u);
        r = (uint32_t)__shfl((int)r, 0, 64);
        if (r >= cap) break;
        blend_tile<STATS>((int)tile_order[x + 8u * r], st, items, dims, ranges, values, geom,
                          conic, rgb, out_single, t_final_all, n_last_all, n_eval_all,
                          n_contrib_all);
        __syncthreads();            // the next tile restages the LDS batch
    }
}

}  // namespace

namespace {
// Workgroups of the persistent blend the GPU holds at once (per device).
template <class K>
int resident_groups(K kernel) {
    static int cached[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (!cached[dev]) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64, 0) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        cached[dev] = per_cu * cus;
    }
    return cached[dev];
}
}  // namespace

hipError_t launch_blend_tiles(const Item* items, const BatchDims& d, const ss_frame& f,
                              const uint32_t* values, float* out_rgb_single, hipStream_t s,
                              bool persistent) {
    const int grid = d.n_tiles;
    if (grid == 0) return hipSuccess;
    const uint32_t* order = tile_order_of(f.table, d.n_items);
    const float4* g4 = reinterpret_cast<const float4*>(f.geom);
    const float4* c4 = reinterpret_cast<const float4*>(f.conic);
    const float4* r4 = reinterpret_cast<const float4*>(f.rgb);
    if (persistent) {
        auto kernel = f.n_eval ? k_blend_persistent<true> : k_blend_persistent<false>;
        const int held = resident_groups(kernel) / 8 * 8;
        const int tiles8 = (grid + 7) / 8 * 8;
        const int pg = held > 0 && held < tiles8 ? held : tiles8;
        hipLaunchKernelGGL(kernel, dim3(pg), dim3(64), 0, s, items, d, order,
                           tile_queue_of(f.table, d.n_items, d.n_tiles), f.ranges, values, g4,
                           c4, r4, out_rgb_single, f.t_final, f.n_last, f.n_eval, f.n_contrib);
        return hipGetLastError();
    }
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(64), 0, s, items, d, order, f.ranges, values,
                           g4, c4, r4, out_rgb_single, f.t_final, f.n_last, f.n_eval,
                           f.n_contrib);
    };
    if (f.n_eval) go(k_blend<true>);
    else go(k_blend<false>);
    return hipGetLastError();
}

hipError_t launch_blend(const Item* items, const BatchDims& d, const ss_frame& f,
                        const uint32_t* values, float* out_rgb_single, hipStream_t s,
                        bool persistent) {
    const hipError_t e = launch_tile_order(items, d, f, s);
    if (e != hipSuccess) return e;
    return launch_blend_tiles(items, d, f, values, out_rgb_single, s, persistent);
}

}  // namespace ss

// Stage 6: per-tile front-to-back alpha blending (Speedy-Splat Sec. 3.3,
// Eqs. render_alpha, 2d_gaussian_scalar and contribution).
//
// One wave (64 lanes) per 16x16 tile.  Lane l owns column l % 16 and rows
// l / 16 + 4s of the four 16x4 strips s = 0..3, so the dx-dependent terms of
// q are computed once per lane and Gaussian and shared by its four pixels, and
// each strip skips a Gaussian as a unit when none of its 64 pixels lies inside
// the ellipse.  The tile's sorted Gaussians are staged through LDS 64 at a
// time (one record per lane, gathered by index), and the walk ends as soon as
// a ballot finds every pixel of the tile finished.  The quadratic form is
// evaluated as ((a dx) dx + (c dy) dy) + ((2b) dx) dy without contraction and
// compared with the record's t, so the inclusion test (alpha >= 1/255) is
// exact and reproducible.  Nothing on this path is a dense contraction, so it
// runs on the FP32 VALU.
#include "ss_internal.h"

namespace ss {
namespace {

constexpr int kBatch = 64;

__global__ __launch_bounds__(64) void k_blend(int tx_n, int n_tiles, int W, int H, float bg0,
                                              float bg1, float bg2,
                                              const uint32_t* __restrict__ ranges,
                                              const uint32_t* __restrict__ values,
                                              const float4* __restrict__ geom,
                                              const float4* __restrict__ conic,
                                              const float4* __restrict__ rgb,
                                              float* __restrict__ out,
                                              float* __restrict__ t_final,
                                              uint32_t* __restrict__ n_last,
                                              uint32_t* __restrict__ n_eval) {
    __shared__ float4 s_geo[kBatch];   // (u, v, -, t)
    __shared__ float4 s_con[kBatch];   // (a, 2b, c, sigma)
    __shared__ float4 s_col[kBatch];   // (r, g, b, -)
    const int tile = xcd_contiguous((int)blockIdx.x, n_tiles);
    if (tile < 0) return;
    const int lane = (int)threadIdx.x;
    const int tx = tile % tx_n, ty = tile / tx_n;
    const int px = tx * kTile + (lane & 15);
    const int py0 = ty * kTile + (lane >> 4);
    const float fx = (float)px + 0.5f;
    float fy[4], T[4], C[4][3];
    uint32_t last[4], stop[4];
    bool alive[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        fy[s] = (float)(py0 + 4 * s) + 0.5f;
        T[s] = 1.0f;
        C[s][0] = C[s][1] = C[s][2] = 0.0f;
        last[s] = 0u;
        stop[s] = 0u;
        alive[s] = px < W && (py0 + 4 * s) < H;
    }
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
    bool any = __ballot(alive[0] | alive[1] | alive[2] | alive[3]) != 0ull;
    for (uint32_t base = start; base < end && any; base += kBatch) {
        const uint32_t j = base + lane;
        if (j < end) {
            const uint32_t gi = values[j];
            const float4 g = geom[gi], q = conic[gi];
            s_geo[lane] = g;
            s_con[lane] = make_float4(q.x, 2.0f * q.y, q.z, q.w);
            s_col[lane] = rgb[gi];
        }
        __syncthreads();
        const uint32_t nb = end - base < (uint32_t)kBatch ? end - base : (uint32_t)kBatch;
        for (uint32_t k = 0; k < nb; ++k) {
            const float4 g = s_geo[k];
            const float4 q = s_con[k];
            const float dx = fx - g.x;
            const float adx2 = (q.x * dx) * dx;
            const float b2dx = q.y * dx;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const float dy = fy[s] - g.y;
                const float qq = (adx2 + (q.z * dy) * dy) + b2dx * dy;
                if (alive[s] && qq <= g.w) {
                    const float al = fminf(kAlphaMax, q.w * __expf(-0.5f * qq));
                    const float tn = T[s] * (1.0f - al);
                    if (tn < kTMin) {
                        alive[s] = false;
                        stop[s] = base + k - start + 1u;
                    } else {
                        const float4 c = s_col[k];
                        const float w = al * T[s];
                        C[s][0] = fmaf(c.x, w, C[s][0]);
                        C[s][1] = fmaf(c.y, w, C[s][1]);
                        C[s][2] = fmaf(c.z, w, C[s][2]);
                        T[s] = tn;
                        last[s] = base + k - start + 1u;
                    }
                }
            }
            if (__ballot(alive[0] | alive[1] | alive[2] | alive[3]) == 0ull) {
                any = false;
                break;
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
            if (n_eval) n_eval[p] = alive[s] ? end - start : stop[s];
        }
    }
}

}  // namespace

hipError_t launch_blend(const ss_camera& cam, const ss_frame& f, const uint32_t* values,
                        float* out_rgb, hipStream_t s) {
    const int tx_n = (cam.width + kTile - 1) / kTile, ty_n = (cam.height + kTile - 1) / kTile;
    const int n_tiles = tx_n * ty_n;
    const int grid = 8 * ((n_tiles + 7) / 8);
    hipLaunchKernelGGL(k_blend, dim3(grid), dim3(64), 0, s, tx_n, n_tiles, cam.width, cam.height,
                       cam.bg[0], cam.bg[1], cam.bg[2], f.ranges, values,
                       reinterpret_cast<const float4*>(f.geom),
                       reinterpret_cast<const float4*>(f.conic),
                       reinterpret_cast<const float4*>(f.rgb), out_rgb, f.t_final, f.n_last,
                       f.n_eval);
    return hipGetLastError();
}

}  // namespace ss

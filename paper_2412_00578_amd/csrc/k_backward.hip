// Adjoint of the forward render: the gradient flow of Speedy-Splat Sec. 4.2
// (per-pixel gradients aggregated to the 2D parameters, then per Gaussian to
// the 3D parameters).
//
// Stage 7, blend backward.  Same tile / strip / wave layout as the forward
// blend.  Each wave walks its tile's list back to front from the last
// Gaussian any of its pixels blended (n_last), recomputing alpha and the
// transmittance before each Gaussian as T_before = T_after / (1 - alpha) from
// the stored final T (no per-pixel, per-Gaussian state is kept from the
// forward pass).  With R the colour of everything behind the Gaussian
// (starting at the background),
//   dC/dc_i     = alpha_i T_i
//   dC/dalpha_i = T_i (c_i - R),   R <- alpha_i c_i + (1 - alpha_i) R.
// The per-pixel gradients with respect to (u, v, a, b, c, sigma, r, g, b) are
// summed over the wave by one transposing reduction that leaves each sum in
// its own lane, and added with one atomic instruction per wave and Gaussian.
// An optional per-Gaussian score accumulates sum over pixels and channels of
// (dC/dg_i)^2, g_i the 2D Gaussian's value at the pixel (the efficient
// pruning score of Sec. 4.2).
//
// Stage 8, preprocess backward.  One lane per Gaussian: the chain rule from
// (u, v, conic, sigma, colour) back to means, scales, quaternions, opacity and
// SH coefficients, with the forward geometry recomputed in FP64.
#include "ss_internal.h"

namespace ss {
namespace {

constexpr int kBatch = 64;
constexpr float kNegHalfLog2e = -0.72134752044448170368f;  // -log2(e) / 2

// The value x of the lane the DPP control names (within a row of 16 lanes).
template <int CTRL>
__device__ __forceinline__ float dpp_pull(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf,
                                                      false));
}

// One halving step of a transposing reduction: lanes pair up through the DPP
// control CTRL, the lane whose bit is set keeps the upper half of the slots,
// its partner the lower half, and each adds the partner's copy of the half it
// keeps.  Slots past N are zero.
template <int CTRL, int N>
__device__ __forceinline__ void halve(const float (&in)[N], float (&out)[(N + 1) / 2], bool up) {
    constexpr int H = (N + 1) / 2;
#pragma unroll
    for (int j = 0; j < H; ++j) {
        const float lo = in[j];
        const float hi = j + H < N ? in[j + H] : 0.0f;
        out[j] = (up ? hi : lo) + dpp_pull<CTRL>(up ? lo : hi);
    }
}

// Wave sums of 10 per-lane values with 35 vector operations instead of 10
// separate 6-step sums.  Within each 16-lane row, four halving steps pair lane
// i with 15 - i (row_mirror), then with its mirror inside the 8-lane half
// (row_half_mirror), then with i ^ 2 and i ^ 1 (quad_perm): partners always
// hold the same slots, and every step halves the slots a lane keeps, so lane
// i ends with the row sum of one value.  Two cross-row swaps (lanes i ^ 16,
// i ^ 32) complete the sums.  Lane l then holds the wave sum of value
// sum10_slot(l & 15), or nothing when that is negative.
__device__ __forceinline__ float wave_sum10(const float (&v)[10], int lane) {
    float a[5], b[3], c[2], d[1];
    halve<0x140, 10>(v, a, (lane & 8) != 0);   // row_mirror
    halve<0x141, 5>(a, b, (lane & 4) != 0);    // row_half_mirror
    halve<0x4E, 3>(b, c, (lane & 2) != 0);     // quad_perm [2, 3, 0, 1]
    halve<0xB1, 2>(c, d, (lane & 1) != 0);     // quad_perm [1, 0, 3, 2]
    float x = d[0];
    x += __shfl_xor(x, 16, 64);
    x += __shfl_xor(x, 32, 64);
    return x;
}

// The value whose sum wave_sum10 leaves in lanes with (l & 15) == r, or -1.
__host__ __device__ constexpr int sum10_slot(int r) {
    const int s3 = r & 1;
    const int s2 = (r & 2) ? s3 + 2 : s3;
    const int s1 = (r & 4) ? s2 + 3 : s2;
    return s2 >= 3 || s1 >= 5 ? -1 : ((r & 8) ? s1 + 5 : s1);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const uint32_t y = __shfl_xor(x, m, 64);
        x = y > x ? y : x;
    }
    return x;
}

// Bit s: the Gaussian's ellipse box, widened by 1% (far more than the FP64
// rounding of q for a conic whose eigenvalue ratio is bounded as tested), meets
// strip s of tile (tx, ty).  Pixel centres outside the box never pass q <= t,
// so a Gaussian whose mask misses every strip of the wave is skipped whole.
__device__ __forceinline__ uint32_t strip_mask_b(float4 g, float4 q, int tx, int ty) {
    const double a = q.x, b = q.y, c = q.z, t = g.w;
    const double det = a * c - b * b;
    if (!(t > 0.0)) return t == 0.0 ? 0xFu : 0u;
    if (!(det > 0.0) || (a + c) * (a + c) > 1.0e3 * det) return 0xFu;
    const double hx = 1.01 * sqrt((t * c) / det) + 1e-3;
    const double hy = 1.01 * sqrt((t * a) / det) + 1e-3;
    const double u = g.x, v = g.y;
    const double x0 = 16.0 * tx + 0.5, x1 = 16.0 * tx + 15.5;
    if (x1 < u - hx || x0 > u + hx) return 0u;
    uint32_t m = 0u;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const double y0 = 16.0 * ty + 4.0 * s + 0.5, y1 = y0 + 3.0;
        if (!(y1 < v - hy || y0 > v + hy)) m |= 1u << s;
    }
    return m;
}

template <int SPW, bool SCORE>
__global__ __launch_bounds__(64 * (4 / SPW)) void k_blend_bwd(
    int tx_n, int n_tiles, int W, int H, float bg0, float bg1, float bg2,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ values,
    const float4* __restrict__ geom, const float4* __restrict__ conic,
    const float4* __restrict__ rgb, const float* __restrict__ t_final,
    const uint32_t* __restrict__ n_last, const float* __restrict__ dl_drgb,
    float* __restrict__ g2d, float* __restrict__ score) {
    constexpr int kWaves = 4 / SPW;
    __shared__ double2 s_uv[kWaves][kBatch];   // (u, v)
    __shared__ double2 s_ab[kWaves][kBatch];   // (a, 2b)
    __shared__ double2 s_ct[kWaves][kBatch];   // (c, t)
    __shared__ float4 s_col[kWaves][kBatch];   // (r, g, b, sigma)
    __shared__ uint32_t s_mask[kWaves][kBatch];  // strip mask bits
    __shared__ uint32_t s_idx[kWaves][kBatch];
    const int tile = xcd_contiguous((int)blockIdx.x, n_tiles);
    if (tile < 0) return;
    const int w = (int)(threadIdx.x >> 6);
    const int lane = (int)(threadIdx.x & 63);
    const int strip0 = w * SPW;
    const int tx = tile % tx_n, ty = tile / tx_n;
    const int px = tx * kTile + (lane & 15);
    const int py0 = ty * kTile + 4 * strip0 + (lane >> 4);
    const double fx = (double)px + 0.5;
    const size_t hw = (size_t)W * (size_t)H;
    double fy[SPW];
    float T[SPW], R[SPW][3], dC[SPW][3];
    uint32_t nl[SPW];
    uint32_t jmax = 0u;
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
        const int py = py0 + 4 * s;
        fy[s] = (double)py + 0.5;
        const bool in = px < W && py < H;
        const size_t p = in ? (size_t)py * W + px : 0;
        nl[s] = in ? n_last[p] : 0u;
        T[s] = in ? t_final[p] : 1.0f;
        R[s][0] = bg0; R[s][1] = bg1; R[s][2] = bg2;
        dC[s][0] = in ? dl_drgb[p] : 0.0f;
        dC[s][1] = in ? dl_drgb[hw + p] : 0.0f;
        dC[s][2] = in ? dl_drgb[2 * hw + p] : 0.0f;
        jmax = nl[s] > jmax ? nl[s] : jmax;
    }
    jmax = wave_max_u32(jmax);
    // the per-Gaussian sums land one per lane in lanes 0..15 (wave_sum10)
    const int red_slot = lane < 16 ? sum10_slot(lane) : -1;
    // g2d row offsets of (u, v, a, b, c, sigma, r, g, b): 0, 1, 4 .. 10
    const int red_off = red_slot < 2 ? red_slot : red_slot + 2;
    const uint32_t start = ranges[2 * tile];
    for (uint32_t hi = jmax; hi > 0u;) {
        const uint32_t lo = hi > (uint32_t)kBatch ? hi - kBatch : 0u;
        const uint32_t cnt = hi - lo;
        if ((uint32_t)lane < cnt) {
            const uint32_t gi = values[start + lo + lane];
            const float4 g = geom[kRec * (size_t)gi], q = conic[kRec * (size_t)gi], c = rgb[gi];
            s_uv[w][lane] = make_double2(g.x, g.y);
            s_ab[w][lane] = make_double2(q.x, 2.0 * (double)q.y);
            s_ct[w][lane] = make_double2(q.z, g.w);
            s_col[w][lane] = make_float4(c.x, c.y, c.z, q.w);
            s_mask[w][lane] = strip_mask_b(g, q, tx, ty);
            s_idx[w][lane] = gi;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int k = (int)cnt - 1; k >= 0; --k) {
            const uint32_t j = lo + (uint32_t)k;
            uint32_t m = __builtin_amdgcn_readfirstlane(s_mask[w][k]);
            if (!(m & (((1u << SPW) - 1u) << strip0))) continue;
            const double2 uv = s_uv[w][k];
            const double2 ab = s_ab[w][k];
            const double2 ct = s_ct[w][k];
            const float4 c = s_col[w][k];
            // the forward's inclusion test, bit for bit (FP64 on the record)
            const double dx64 = fx - uv.x;
            const double adx2 = (ab.x * dx64) * dx64;
            const double b2dx = ab.y * dx64;
            const float dx = (float)dx64;
            const float qa = (float)ab.x, qb2 = (float)ab.y, qc = (float)ct.x, sig = c.w;
            float gu = 0.f, gv = 0.f, ga = 0.f, gb = 0.f, gc = 0.f, gs = 0.f;
            float gr = 0.f, gg = 0.f, gbl = 0.f, sc = 0.f;
            bool any = false;
#pragma unroll
            for (int s = 0; s < SPW; ++s) {
                const double dy64 = fy[s] - uv.y;
                const double q64 = fma(fma(ct.x, dy64, b2dx), dy64, adx2);
                if (j < nl[s] && q64 <= ct.y) {
                    any = true;
                    const float qq = (float)q64, dy = (float)dy64;
                    const float gval = __builtin_amdgcn_exp2f(qq * kNegHalfLog2e);  // exp(-q/2)
                    const float araw = sig * gval;
                    const float al = fminf(kAlphaMax, araw);
                    // hardware reciprocal (about 1 ulp): the recurrence runs over the
                    // pixel's blended Gaussians only, well inside the gradients' tolerance
                    const float tb = T[s] * __builtin_amdgcn_rcpf(1.0f - al);
                    const float wgt = al * tb;
                    gr = fmaf(wgt, dC[s][0], gr);
                    gg = fmaf(wgt, dC[s][1], gg);
                    gbl = fmaf(wgt, dC[s][2], gbl);
                    const float e0 = c.x - R[s][0], e1 = c.y - R[s][1], e2 = c.z - R[s][2];
                    const float dal = tb * (dC[s][0] * e0 + dC[s][1] * e1 + dC[s][2] * e2);
                    R[s][0] = fmaf(al, c.x, (1.0f - al) * R[s][0]);
                    R[s][1] = fmaf(al, c.y, (1.0f - al) * R[s][1]);
                    R[s][2] = fmaf(al, c.z, (1.0f - al) * R[s][2]);
                    T[s] = tb;
                    // a clamped alpha passes no gradient to q and sigma
                    const float dau = araw < kAlphaMax ? dal : 0.0f;
                    gs = fmaf(dau, gval, gs);
                    const float dq = -0.5f * al * dau;
                    // q = a dx^2 + 2b dx dy + c dy^2 with dx = px - u, dy = py - v
                    gu += dq * -(2.0f * qa * dx + qb2 * dy);
                    gv += dq * -(qb2 * dx + 2.0f * qc * dy);
                    ga = fmaf(dq, dx * dx, ga);
                    gb = fmaf(dq, 2.0f * dx * dy, gb);
                    gc = fmaf(dq, dy * dy, gc);
                    if (SCORE) {
                        const float k0 = araw < kAlphaMax ? sig * tb : 0.0f;
                        sc += k0 * k0 * (e0 * e0 + e1 * e1 + e2 * e2);
                    }
                }
            }
            if (__ballot(any) == 0ull) continue;
            const float part[10] = {gu, gv, ga, gb, gc, gs, gr, gg, gbl, sc};
            const float tot = wave_sum10(part, lane);
            if (red_slot >= 0) {
                const uint32_t gi = s_idx[w][k];
                if (red_slot < 9) atomicAdd(g2d + (size_t)gi * 12 + red_off, tot);
                else if (SCORE) atomicAdd(score + gi, tot);
            }
        }
        __builtin_amdgcn_wave_barrier();
        hi = lo;
    }
}

__global__ void k_fill_zero(float* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// ------------------------------------------------------------ preprocess backward

// Real SH constants (degrees 0..3, Condon-Shortley phase), as in the forward.
constexpr float kC0 = 0.28209479177387814f;
constexpr float kC1 = 0.4886025119029199f;
constexpr float kC2a = 1.0925484305920792f, kC2b = 0.31539156525252005f,
                kC2c = 0.5462742152960396f;
constexpr float kC3a = 0.5900435899266435f, kC3b = 2.890611442640554f,
                kC3c = 0.4570457994644658f, kC3d = 0.3731763325901154f,
                kC3e = 1.445305721320277f;

// Basis function k and its partial derivatives with respect to the direction
// components (x, y, z), at a unit direction; k is a compile-time constant in
// the unrolled callers, so no table is materialised.
__device__ __forceinline__ void sh_term(int k, float x, float y, float z, float& Y, float& gx,
                                        float& gy, float& gz) {
    const float xx = x * x, yy = y * y, zz = z * z;
    gx = gy = gz = 0.0f;
    switch (k) {
        case 0: Y = kC0; break;
        case 1: Y = -kC1 * y; gy = -kC1; break;
        case 2: Y = kC1 * z; gz = kC1; break;
        case 3: Y = -kC1 * x; gx = -kC1; break;
        case 4: Y = kC2a * x * y; gx = kC2a * y; gy = kC2a * x; break;
        case 5: Y = -kC2a * y * z; gy = -kC2a * z; gz = -kC2a * y; break;
        case 6: Y = kC2b * (2.0f * zz - xx - yy);
                gx = -2.0f * kC2b * x; gy = -2.0f * kC2b * y; gz = 4.0f * kC2b * z; break;
        case 7: Y = -kC2a * x * z; gx = -kC2a * z; gz = -kC2a * x; break;
        case 8: Y = kC2c * (xx - yy); gx = 2.0f * kC2c * x; gy = -2.0f * kC2c * y; break;
        case 9: Y = -kC3a * y * (3.0f * xx - yy);
                gx = -6.0f * kC3a * x * y; gy = -kC3a * (3.0f * xx - 3.0f * yy); break;
        case 10: Y = kC3b * x * y * z; gx = kC3b * y * z; gy = kC3b * x * z; gz = kC3b * x * y;
                 break;
        case 11: Y = -kC3c * y * (4.0f * zz - xx - yy);
                 gx = 2.0f * kC3c * x * y; gy = -kC3c * (4.0f * zz - xx - 3.0f * yy);
                 gz = -8.0f * kC3c * y * z; break;
        case 12: Y = kC3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
                 gx = -6.0f * kC3d * x * z; gy = -6.0f * kC3d * y * z;
                 gz = kC3d * (6.0f * zz - 3.0f * xx - 3.0f * yy); break;
        case 13: Y = -kC3c * x * (4.0f * zz - xx - yy);
                 gx = -kC3c * (4.0f * zz - 3.0f * xx - yy); gy = 2.0f * kC3c * x * y;
                 gz = -8.0f * kC3c * x * z; break;
        case 14: Y = kC3e * z * (xx - yy); gx = 2.0f * kC3e * x * z; gy = -2.0f * kC3e * y * z;
                 gz = kC3e * (xx - yy); break;
        default: Y = -kC3a * x * (xx - 3.0f * yy); gx = -kC3a * (3.0f * xx - 3.0f * yy);
                 gy = 6.0f * kC3a * x * y; break;
    }
}

struct BwdIn {
    const float* means;
    const float* scales;
    const float* quats;
    const float* opacity;
    const float* sh;
    int sh_degree, sh_stride;
};

struct BwdOut {
    float* means;
    float* scales;
    float* quats;
    float* opacity;
    float* sh;
};

constexpr int kPbBlock = 64;               // one wave per workgroup
constexpr int kShRow = 48;                 // SH floats per Gaussian staged (degree 3)
constexpr int kShPitchB = kShRow + 1;      // odd LDS pitch

// Stage 8.  One lane per Gaussian, one wave per workgroup.  The SH part runs
// in FP32 (the forward colour is FP32).  ROWS (every SH row 16-byte aligned):
// a lane whose colour passes a gradient loads its own row into registers with
// up to 12 16-byte loads (the others read nothing), and the wave's dL/dh rows,
// zeros for the others, are staged through LDS and stored coalesced (per-lane
// row stores scatter each store instruction over 64 rows: the kernel took
// 0.21 ms that way, 0.12 ms now).  Otherwise the workgroup's SH rows are staged
// through LDS with coalesced loads, each lane overwrites its row in place with
// dL/dh, and the rows are written back coalesced.  The geometry chain is FP64.
template <bool ROWS>
__global__ __launch_bounds__(kPbBlock) void k_preprocess_bwd(ss_camera cam, BwdIn in, int64_t n,
                                                            const float4* __restrict__ conic_rec,
                                                            const float4* __restrict__ rgb_rec,
                                                            const float* __restrict__ g2d,
                                                            BwdOut out) {
    const int64_t first = (int64_t)blockIdx.x * kPbBlock;
    const int64_t i = first + threadIdx.x;
    const int nb = (in.sh_degree + 1) * (in.sh_degree + 1);
    const int need = 3 * nb, row = 3 * in.sh_stride;
    const bool real = i < n;
    const float4 rec = real ? conic_rec[kRec * i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const bool alive = rec.x != 0.0f || rec.y != 0.0f || rec.z != 0.0f;
    const float* G = g2d + (size_t)(real ? i : 0) * 12;
    const float4 col = real ? rgb_rec[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    // a channel the forward clamped to 0, as its stored colour shows, passes no gradient
    const float gs0 = alive && col.x > 0.0f ? G[8] : 0.0f;
    const float gs1 = alive && col.y > 0.0f ? G[9] : 0.0f;
    const float gs2 = alive && col.z > 0.0f ? G[10] : 0.0f;

    // ---- colour -> SH and view direction (FP32)
    float gdx = 0.0f, gdy = 0.0f, gdz = 0.0f, dirx = 0.0f, diry = 0.0f, dirz = 0.0f, len = 1.0f;
    if (real) {
        const float cpx = -((cam.R[0] * cam.t[0] + cam.R[3] * cam.t[1]) + cam.R[6] * cam.t[2]);
        const float cpy = -((cam.R[1] * cam.t[0] + cam.R[4] * cam.t[1]) + cam.R[7] * cam.t[2]);
        const float cpz = -((cam.R[2] * cam.t[0] + cam.R[5] * cam.t[1]) + cam.R[8] * cam.t[2]);
        const float dvx = in.means[3 * i] - cpx, dvy = in.means[3 * i + 1] - cpy,
                    dvz = in.means[3 * i + 2] - cpz;
        len = sqrtf(dvx * dvx + dvy * dvy + dvz * dvz);
        dirx = dvx / len; diry = dvy / len; dirz = dvz / len;
    }
    if constexpr (ROWS) {
        const int q = (need + 3) / 4;            // 16-byte pieces holding the coefficients
        const bool grad = real && (gs0 != 0.0f || gs1 != 0.0f || gs2 != 0.0f);
        float h[48];
#pragma unroll
        for (int k = 0; k < 48; ++k) h[k] = 0.0f;
        if (grad) {
            const float4* src = reinterpret_cast<const float4*>(in.sh + i * row);
            float4 v[12];
#pragma unroll
            for (int j = 0; j < 12; ++j) v[j] = j < q ? src[j] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int j = 0; j < 12; ++j) {
                h[4 * j] = v[j].x; h[4 * j + 1] = v[j].y; h[4 * j + 2] = v[j].z;
                h[4 * j + 3] = v[j].w;
            }
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                if (k < nb) {
                    float Y, tx, ty, tz;
                    sh_term(k, dirx, diry, dirz, Y, tx, ty, tz);
                    const float gy = (h[3 * k] * gs0 + h[3 * k + 1] * gs1) + h[3 * k + 2] * gs2;
                    gdx = fmaf(gy, tx, gdx);
                    gdy = fmaf(gy, ty, gdy);
                    gdz = fmaf(gy, tz, gdz);
                    h[3 * k] = Y * gs0;
                    h[3 * k + 1] = Y * gs1;
                    h[3 * k + 2] = Y * gs2;
                }
            }
#pragma unroll
            for (int k = 0; k < 48; ++k)
                if (k >= need) h[k] = 0.0f;          // the row's floats past the coefficients
        }
        // the wave's rows are contiguous: stage them in LDS and store them
        // with consecutive lanes on consecutive 16-byte pieces
        __shared__ float4 s_out[kPbBlock * 12];
#pragma unroll
        for (int j = 0; j < 12; ++j)
            s_out[threadIdx.x * 12 + j] = make_float4(h[4 * j], h[4 * j + 1], h[4 * j + 2],
                                                      h[4 * j + 3]);
        __syncthreads();
        const int cnt = n - first < kPbBlock ? (int)(n - first) : kPbBlock;
        const int row4 = row / 4;                // at most 12 pieces per row here
        float4* dst = reinterpret_cast<float4*>(out.sh + first * row);
        for (int c = threadIdx.x; c < cnt * row4; c += kPbBlock) {
            const int g = c / row4;
            dst[c] = s_out[g * 12 + (c - g * row4)];
        }
    } else {
        __shared__ float s_h[kPbBlock * kShPitchB];
        const int cnt = n - first < kPbBlock ? (int)(n - first) : kPbBlock;
        for (int e = threadIdx.x; e < cnt * need; e += kPbBlock) {
            const int g = e / need, j = e - g * need;
            s_h[g * kShPitchB + j] = in.sh[(first + g) * row + j];
        }
        __syncthreads();
        float* h = s_h + threadIdx.x * kShPitchB;
        if (real && !(gs0 != 0.0f || gs1 != 0.0f || gs2 != 0.0f)) {
            for (int k = 0; k < need; ++k) h[k] = 0.0f;   // no colour gradient: dL/dh = 0
        } else if (real) {
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                if (k < nb) {
                    float Y, tx, ty, tz;
                    sh_term(k, dirx, diry, dirz, Y, tx, ty, tz);
                    const float gy = (h[3 * k] * gs0 + h[3 * k + 1] * gs1) + h[3 * k + 2] * gs2;
                    gdx = fmaf(gy, tx, gdx);
                    gdy = fmaf(gy, ty, gdy);
                    gdz = fmaf(gy, tz, gdz);
                    h[3 * k] = Y * gs0;            // dL/dh replaces h in this lane's own row
                    h[3 * k + 1] = Y * gs1;
                    h[3 * k + 2] = Y * gs2;
                }
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < cnt * row; e += kPbBlock) {
            const int g = e / row, j = e - g * row;
            out.sh[(first + g) * row + j] = j < need ? s_h[g * kShPitchB + j] : 0.0f;
        }
    }
    if (!real) return;
    if (!alive) {
        for (int k = 0; k < 3; ++k) { out.means[3 * i + k] = 0.f; out.scales[3 * i + k] = 0.f; }
        for (int k = 0; k < 4; ++k) out.quats[4 * i + k] = 0.f;
        out.opacity[i] = 0.f;
        return;
    }
    const double gu = G[0], gv = G[1], ga = G[4], gb = G[5], gc = G[6];
    out.opacity[i] = G[7];

    const double Rc[9] = {cam.R[0], cam.R[1], cam.R[2], cam.R[3], cam.R[4],
                          cam.R[5], cam.R[6], cam.R[7], cam.R[8]};
    const double mx = in.means[3 * i], my = in.means[3 * i + 1], mz = in.means[3 * i + 2];
    const double x = ((Rc[0] * mx + Rc[1] * my) + Rc[2] * mz) + (double)cam.t[0];
    const double y = ((Rc[3] * mx + Rc[4] * my) + Rc[5] * mz) + (double)cam.t[1];
    const double z = ((Rc[6] * mx + Rc[7] * my) + Rc[8] * mz) + (double)cam.t[2];
    const double fx = cam.fx, fy = cam.fy;
    double gpos[3] = {0.0, 0.0, 0.0};   // gradient w.r.t. the camera-space point
    double gmean[3];                    // gradient w.r.t. the world mean
    {   // the view direction d = v / |v|, v = mean - camera centre
        const float dd = (gdx * dirx + gdy * diry) + gdz * dirz;
        gmean[0] = (double)((gdx - dirx * dd) / len);
        gmean[1] = (double)((gdy - diry * dd) / len);
        gmean[2] = (double)((gdz - dirz * dd) / len);
    }

    // ---- projection of the mean
    gpos[0] += gu * fx / z;
    gpos[1] += gv * fy / z;
    gpos[2] += -gu * fx * x / (z * z) - gv * fy * y / (z * z);

    // ---- forward geometry (FP64) for the covariance chain
    const float4 qr = *reinterpret_cast<const float4*>(in.quats + 4 * i);
    const double q0 = qr.x, q1 = qr.y, q2 = qr.z, q3 = qr.w;
    const double qnorm = sqrt(((q0 * q0 + q1 * q1) + q2 * q2) + q3 * q3);
    const double w_ = q0 / qnorm, x_ = q1 / qnorm, y_ = q2 / qnorm, z_ = q3 / qnorm;
    double Rq[9];
    Rq[0] = 1.0 - 2.0 * (y_ * y_ + z_ * z_);
    Rq[1] = 2.0 * (x_ * y_ - w_ * z_);
    Rq[2] = 2.0 * (x_ * z_ + w_ * y_);
    Rq[3] = 2.0 * (x_ * y_ + w_ * z_);
    Rq[4] = 1.0 - 2.0 * (x_ * x_ + z_ * z_);
    Rq[5] = 2.0 * (y_ * z_ - w_ * x_);
    Rq[6] = 2.0 * (x_ * z_ - w_ * y_);
    Rq[7] = 2.0 * (y_ * z_ + w_ * x_);
    Rq[8] = 1.0 - 2.0 * (x_ * x_ + y_ * y_);
    const double sc[3] = {in.scales[3 * i], in.scales[3 * i + 1], in.scales[3 * i + 2]};
    double M[9], S3[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) M[3 * r + c] = Rq[3 * r + c] * sc[c];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            S3[3 * r + c] = M[3 * r] * M[3 * c] + M[3 * r + 1] * M[3 * c + 1] + M[3 * r + 2] * M[3 * c + 2];
    const double limx = kFovClamp * ((0.5 * (double)cam.width) / fx);
    const double limy = kFovClamp * ((0.5 * (double)cam.height) / fy);
    const double rx = x / z, ry = y / z;
    const bool clx = rx < -limx || rx > limx, cly = ry < -limy || ry > limy;
    const double txz = rx < -limx ? -limx : (rx > limx ? limx : rx);
    const double tyz = ry < -limy ? -limy : (ry > limy ? limy : ry);
    const double J00 = fx / z, J02 = -(fx * txz) / z, J11 = fy / z, J12 = -(fy * tyz) / z;
    double T[6];
    for (int j = 0; j < 3; ++j) {
        T[j] = J00 * Rc[j] + J02 * Rc[6 + j];
        T[3 + j] = J11 * Rc[3 + j] + J12 * Rc[6 + j];
    }
    double V[6];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
            V[3 * r + c] = T[3 * r] * S3[c] + T[3 * r + 1] * S3[3 + c] + T[3 * r + 2] * S3[6 + c];
    const double A = V[0] * T[0] + V[1] * T[1] + V[2] * T[2] + kDilation;
    const double B = V[0] * T[3] + V[1] * T[4] + V[2] * T[5];
    const double C = V[3] * T[3] + V[4] * T[4] + V[5] * T[5] + kDilation;
    const double D = A * C - B * B;
    const double D2 = D * D;

    // ---- conic (a, b, c) = (C, -B, A) / D  ->  (A, B, C)
    const double gA = (-ga * C * C + gb * B * C - gc * B * B) / D2;
    const double gB = (2.0 * ga * B * C - gb * (A * C + B * B) + 2.0 * gc * A * B) / D2;
    const double gC = (-ga * B * B + gb * A * B - gc * A * A) / D2;
    // symmetric upstream gradient of Sigma_2D (B sits in both off-diagonal entries)
    const double G00 = gA, G01 = 0.5 * gB, G11 = gC;

    // ---- Sigma_2D = T Sigma_3D T^T:  gS3 = T^T G T,  gT = 2 G T Sigma_3D
    double GT[6];   // G T (2x3)
    for (int c = 0; c < 3; ++c) {
        GT[c] = G00 * T[c] + G01 * T[3 + c];
        GT[3 + c] = G01 * T[c] + G11 * T[3 + c];
    }
    double gS3[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) gS3[3 * r + c] = T[r] * GT[c] + T[3 + r] * GT[3 + c];
    double gT[6];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
            gT[3 * r + c] = 2.0 * (GT[3 * r] * S3[c] + GT[3 * r + 1] * S3[3 + c] +
                                   GT[3 * r + 2] * S3[6 + c]);
    // T = J Rc:  gJ = gT Rc^T (only J00, J02, J11, J12 vary)
    const double gJ00 = gT[0] * Rc[0] + gT[1] * Rc[1] + gT[2] * Rc[2];
    const double gJ02 = gT[0] * Rc[6] + gT[1] * Rc[7] + gT[2] * Rc[8];
    const double gJ11 = gT[3] * Rc[3] + gT[4] * Rc[4] + gT[5] * Rc[5];
    const double gJ12 = gT[3] * Rc[6] + gT[4] * Rc[7] + gT[5] * Rc[8];
    const double z2 = z * z, z3 = z2 * z;
    gpos[2] += -gJ00 * fx / z2 - gJ11 * fy / z2;
    if (!clx) {
        gpos[0] += -gJ02 * fx / z2;
        gpos[2] += gJ02 * 2.0 * fx * x / z3;
    } else {
        gpos[2] += gJ02 * fx * txz / z2;
    }
    if (!cly) {
        gpos[1] += -gJ12 * fy / z2;
        gpos[2] += gJ12 * 2.0 * fy * y / z3;
    } else {
        gpos[2] += gJ12 * fy * tyz / z2;
    }
    // camera space -> world
    for (int a = 0; a < 3; ++a)
        gmean[a] += Rc[a] * gpos[0] + Rc[3 + a] * gpos[1] + Rc[6 + a] * gpos[2];
    for (int a = 0; a < 3; ++a) out.means[3 * i + a] = (float)gmean[a];

    // ---- Sigma_3D = M M^T, M = Rq diag(s)
    double gM[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            gM[3 * r + c] = 2.0 * (gS3[3 * r] * M[c] + gS3[3 * r + 1] * M[3 + c] +
                                   gS3[3 * r + 2] * M[6 + c]);
    double gRq[9];
    for (int c = 0; c < 3; ++c) {
        double gsc = 0.0;
        for (int r = 0; r < 3; ++r) {
            gsc += gM[3 * r + c] * Rq[3 * r + c];
            gRq[3 * r + c] = gM[3 * r + c] * sc[c];
        }
        out.scales[3 * i + c] = (float)gsc;
    }
    // rotation of the unit quaternion (w, x, y, z)
    double gw = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    gx += -4.0 * x_ * (gRq[4] + gRq[8]);
    gy += -4.0 * y_ * (gRq[0] + gRq[8]);
    gz += -4.0 * z_ * (gRq[0] + gRq[4]);
    gw += 2.0 * (-z_ * gRq[1] + y_ * gRq[2] + z_ * gRq[3] - x_ * gRq[5] - y_ * gRq[6] + x_ * gRq[7]);
    gx += 2.0 * (y_ * gRq[1] + z_ * gRq[2] + y_ * gRq[3] - w_ * gRq[5] + z_ * gRq[6] + w_ * gRq[7]);
    gy += 2.0 * (x_ * gRq[1] + w_ * gRq[2] + x_ * gRq[3] + z_ * gRq[5] - w_ * gRq[6] + z_ * gRq[7]);
    gz += 2.0 * (-w_ * gRq[1] + x_ * gRq[2] + w_ * gRq[3] + y_ * gRq[5] + x_ * gRq[6] + y_ * gRq[7]);
    // through the normalisation q / |q|
    const double dot = gw * w_ + gx * x_ + gy * y_ + gz * z_;
    out.quats[4 * i + 0] = (float)((gw - w_ * dot) / qnorm);
    out.quats[4 * i + 1] = (float)((gx - x_ * dot) / qnorm);
    out.quats[4 * i + 2] = (float)((gy - y_ * dot) / qnorm);
    out.quats[4 * i + 3] = (float)((gz - z_ * dot) / qnorm);
}

}  // namespace

hipError_t launch_backward(const ss_camera& cam, const ss_gaussians& g, const ss_frame& f,
                           const uint32_t* values, const float* dl_drgb, const ss_grads& out,
                           void* const* ev, hipStream_t s) {
    const int tx_n = (cam.width + kTile - 1) / kTile, ty_n = (cam.height + kTile - 1) / kTile;
    const int n_tiles = tx_n * ty_n;
    auto mark = [&](int k) {
        if (ev && ev[k]) (void)hipEventRecord((hipEvent_t)ev[k], s);
    };
    mark(0);
    if (g.n > 0) {
        const int64_t m = g.n * 12;
        hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s,
                           out.g2d, m);
        if (out.score)
            hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((g.n + 255) / 256)), dim3(256), 0, s,
                               out.score, g.n);
    }
    mark(1);
    const int grid = 8 * ((n_tiles + 7) / 8);
    hipLaunchKernelGGL((out.score ? k_blend_bwd<4, true> : k_blend_bwd<4, false>), dim3(grid),
                       dim3(64), 0, s, tx_n, n_tiles, cam.width, cam.height, cam.bg[0],
                       cam.bg[1], cam.bg[2], f.ranges, values,
                       reinterpret_cast<const float4*>(f.geom),
                       reinterpret_cast<const float4*>(f.conic),
                       reinterpret_cast<const float4*>(f.rgb), f.t_final, f.n_last, dl_drgb,
                       out.g2d, out.score);
    mark(2);
    if (g.n > 0) {
        BwdIn in{g.means, g.scales, g.quats, g.opacity, g.sh, g.sh_degree, g.sh_stride};
        BwdOut o{out.means, out.scales, out.quats, out.opacity, out.sh};
        // float4 row loads and stores need both SH arrays 16-byte aligned
        const bool rows = ((uintptr_t)g.sh & 15u) == 0 && ((uintptr_t)out.sh & 15u) == 0 &&
                          ((3 * g.sh_stride) & 3) == 0 && g.sh_stride <= 16;
        hipLaunchKernelGGL(rows ? k_preprocess_bwd<true> : k_preprocess_bwd<false>,
                           dim3((unsigned)((g.n + kPbBlock - 1) / kPbBlock)),
                           dim3(kPbBlock), 0, s, cam, in, g.n,
                           reinterpret_cast<const float4*>(f.conic),
                           reinterpret_cast<const float4*>(f.rgb), out.g2d, o);
    }
    mark(3);
    return hipGetLastError();
}

}  // namespace ss

// Stage 1: per-Gaussian preprocess (Speedy-Splat Sec. 3.2.1, "Preprocessing",
// with the opacity-aware threshold of Sec. 4.1).
//
// One lane per Gaussian.  The screen-space geometry is FP64 over the FP32
// inputs and is rounded once into the FP32 record; the tile count is then an
// FP64 function of the stored record.  A record whose tile rectangle fits 8 x 8
// tiles also stores its tile set as a bit mask, which the emit stage expands;
// the emit stage re-walks the same FP64 function for the others, so counts and
// emitted pairs agree by construction.  A second kernel evaluates the FP32
// colour of the Gaussians with tiles, reading only their SH rows (about half
// of the SH data of a typical frame).
#include "ss_internal.h"

namespace ss {
namespace {

// Real SH basis constants, degrees 0..3, ordered (l, m = -l..l) with the
// Condon-Shortley phase.
constexpr float kSH0 = 0.28209479177387814f;
constexpr float kSH1 = 0.4886025119029199f;
constexpr float kSH2a = 1.0925484305920792f, kSH2b = 0.31539156525252005f,
                kSH2c = 0.5462742152960396f;
constexpr float kSH3a = 0.5900435899266435f, kSH3b = 2.890611442640554f,
                kSH3c = 0.4570457994644658f, kSH3d = 0.3731763325901154f,
                kSH3e = 1.445305721320277f;

__device__ __forceinline__ bool finite_f(float x) { return __builtin_isfinite(x); }

struct Inputs {
    const float* means;
    const float* scales;
    const float* quats;
    const float* opacity;
    const float* sh;
    int sh_degree, sh_stride;
};

constexpr int kBlock = 64;                 // one wave: LDS staging per wave
static_assert(kSlotAlign % kBlock == 0, "a preprocess workgroup must not span two items");
constexpr int kPack = 16;                  // items per table-writing launch (kernel-argument bytes)
struct ItemPack {
    Item it[kPack];
};
constexpr int kShMax = 48;                 // SH floats per Gaussian (degree 3)
constexpr int kShPitch = kShMax + 1;       // odd LDS pitch: lanes hit distinct banks

// Copies the first `need` floats of the SH rows of this workgroup's Gaussians
// whose s_vis flag is set into LDS (Gaussian g at s_sh[g * kShPitch]) with
// coalesced loads: the [n, stride, 3] rows of consecutive Gaussians are
// contiguous.  Rows of Gaussians without tiles are not read.
__device__ __forceinline__ void stage_sh(const float* __restrict__ sh, int64_t first, int64_t n,
                                         int row, int need, const uint32_t* s_vis,
                                         float* s_sh) {
    const int cnt = (n - first) < kBlock ? (int)(n - first) : kBlock;
    const float* src = sh + first * row;
    if (((uintptr_t)src & 15u) == 0 && (row & 3) == 0) {
        // float4 j of a Gaussian covers floats 4j .. 4j + 3, all inside its row
        // (row is a multiple of 4); floats past `need` are not kept
        const unsigned q = (unsigned)(need + 3) >> 2, urow4 = (unsigned)row >> 2;
        const float4* src4 = reinterpret_cast<const float4*>(src);
        // kUnroll loads are issued before the first LDS store, so their
        // latencies overlap instead of adding up
        constexpr unsigned kUnroll = 6;
        const unsigned total = (unsigned)cnt * q;
        for (unsigned e0 = threadIdx.x; e0 < total; e0 += kUnroll * kBlock) {
            float4 v[kUnroll];
            unsigned g[kUnroll], j[kUnroll];
            bool ok[kUnroll];
#pragma unroll
            for (unsigned u = 0; u < kUnroll; ++u) {
                const unsigned e = e0 + u * kBlock;
                g[u] = e / q;
                j[u] = e - g[u] * q;
                ok[u] = e < total && s_vis[g[u]];
                v[u] = ok[u] ? ld_global(src4 + g[u] * urow4 + j[u]) : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (unsigned u = 0; u < kUnroll; ++u) {
                if (!ok[u]) continue;
                float* d = s_sh + g[u] * kShPitch + 4 * j[u];
                d[0] = v[u].x;
                if ((int)(4 * j[u]) + 1 < need) d[1] = v[u].y;
                if ((int)(4 * j[u]) + 2 < need) d[2] = v[u].z;
                if ((int)(4 * j[u]) + 3 < need) d[3] = v[u].w;
            }
        }
    } else {
        for (unsigned e = threadIdx.x; e < (unsigned)(cnt * need); e += kBlock) {
            const unsigned g = e / (unsigned)need, j = e - g * (unsigned)need;
            if (s_vis[g]) s_sh[g * kShPitch + j] = ld_global(src + (int64_t)g * row + j);
        }
    }
}

// The geometry kernel's workgroup: four waves, whose AccuTile bands are dealt
// out together (a wave alone leaves a third of its last chunk's lanes idle).
constexpr int kPreBlock = 256;
static_assert(kSlotAlign % kPreBlock == 0, "a preprocess workgroup must not span two items");

// A record's ellipse as the lanes evaluating its bands read it from LDS.
struct BandRec {
    double u, v, a, b, c, t, det, hx, hy;
    int x0, x1, y0, y1;
    int flags;                 // bit 0: bands are columns; bit 1: the set fits the mask window
    int pad;
};
static_assert(sizeof(BandRec) == 96, "band record layout");

// AccuTile tile sets of the workgroup's lanes with `want` set (records g, q):
// the bands of all those records are dealt out to the workgroup's lanes, 64
// to a wave at a time, each band evaluated on its own (accutile_band), and the
// band counts and, for a record whose rectangle fits the window, the band's
// mask bits are gathered per record with LDS atomics.  Returns the lane's
// count and sets *mask / *origin as rect_tile_set does (all zero for a lane
// without `want`).  Every thread of the workgroup must call it.
__device__ __forceinline__ uint32_t accutile_tile_set_wg(bool want, float4 g, float4 q, int tx_n,
                                                         int ty_n, int by0, int by1,
                                                         BandRec* s_rec, uint32_t* s_incl,
                                                         uint32_t* s_nb, uint32_t* s_cnt,
                                                         uint32_t* s_mask, uint32_t* s_wsum,
                                                         uint64_t* mask, uint32_t* origin) {
    const int t = (int)threadIdx.x;
    const int w = t >> 6, lane = t & 63;
    Ellipse e;
    bool fits = false;
    uint32_t nb = 0;
    *mask = 0ull;
    *origin = 0u;
    if (want && ellipse_setup(g, q, SS_TILE_ACCUTILE, tx_n, ty_n, by0, by1, e)) {
        const bool cols = span_columns(e, SS_TILE_ACCUTILE);
        nb = (uint32_t)(cols ? e.x1 - e.x0 + 1 : e.y1 - e.y0 + 1);
        fits = e.x1 - e.x0 < kSetSide && e.y1 - e.y0 < kSetSide;
        if (fits) *origin = (uint32_t)e.x0 | ((uint32_t)(e.y0 - by0) << 16);
        BandRec& r = s_rec[t];
        r.u = e.u; r.v = e.v; r.a = e.a; r.b = e.b; r.c = e.c; r.t = e.t; r.det = e.det;
        r.hx = e.hx; r.hy = e.hy;
        r.x0 = e.x0; r.x1 = e.x1; r.y0 = e.y0; r.y1 = e.y1;
        r.flags = (cols ? 1 : 0) | (fits ? 2 : 0);
    }
    s_nb[t] = nb;
    s_cnt[t] = 0u;
    s_mask[2 * t] = 0u;
    s_mask[2 * t + 1] = 0u;
    // inclusive prefix sum of the band counts over the workgroup
    uint32_t incl = nb;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)incl, d, 64);
        if (lane >= d) incl += y;
    }
    if (lane == 63) s_wsum[w] = incl;
    __syncthreads();
    for (int k = 0; k < w; ++k) incl += s_wsum[k];
    s_incl[t] = incl;
    __syncthreads();
    const uint32_t total = s_incl[kPreBlock - 1];
    for (uint32_t c0 = (uint32_t)w * 64u; c0 < total; c0 += kPreBlock) {   // wave-uniform
        const uint32_t j = c0 + (uint32_t)lane;
        if (j >= total) continue;
        // owner L: the first lane whose inclusive sum exceeds j
        int L = 0;
#pragma unroll
        for (int step = kPreBlock / 2; step >= 1; step >>= 1)
            if (s_incl[L + step - 1] <= j) L += step;
        const int k = (int)(j - (s_incl[L] - s_nb[L]));
        const BandRec& r = s_rec[L];
        Ellipse el;
        el.u = r.u; el.v = r.v; el.a = r.a; el.b = r.b; el.c = r.c; el.t = r.t; el.det = r.det;
        el.hx = r.hx; el.hy = r.hy;
        el.x0 = r.x0; el.x1 = r.x1; el.y0 = r.y0; el.y1 = r.y1;
        const bool cl = (r.flags & 1) != 0, ft = (r.flags & 2) != 0;
        el.cols = cl;
        int lo, hi;
        if (accutile_band(el, cl, k, tx_n, ty_n, lo, hi)) {
            const uint32_t len = (uint32_t)(hi - lo + 1);
            atomicAdd(&s_cnt[L], len);
            if (ft) {
                // row band: a run of len bits; column band: len bits 8 apart
                const uint64_t bits =
                    cl ? (0x0101010101010101ull >> (8u * (kSetSide - len)))
                             << ((lo - el.y0) * kSetSide + k)
                       : ((1ull << len) - 1ull) << (k * kSetSide + (lo - el.x0));
                if ((uint32_t)bits) atomicOr(&s_mask[2 * L], (uint32_t)bits);
                if ((uint32_t)(bits >> 32)) atomicOr(&s_mask[2 * L + 1], (uint32_t)(bits >> 32));
            }
        }
    }
    __syncthreads();
    if (fits) *mask = (uint64_t)s_mask[2 * t] | ((uint64_t)s_mask[2 * t + 1] << 32);
    return nb ? s_cnt[t] : 0u;
}

__global__ __launch_bounds__(kPreBlock) void k_preprocess(const Item* __restrict__ items,
                                                       BatchDims dims, int mode,
                                                       float4* __restrict__ geom,
                                                       float4* __restrict__ conic,
                                                       uint32_t* __restrict__ counts,
                                                       uint32_t* __restrict__ dkeys,
                                                       uint4* __restrict__ tsets,
                                                       uint32_t* __restrict__ partials,
                                                       Item item0, Item* __restrict__ table_out,
                                                       uint64_t* __restrict__ totals) {
    __shared__ BandRec s_rec[kPreBlock];
    __shared__ uint32_t s_incl[kPreBlock], s_nb[kPreBlock], s_cnt[kPreBlock];
    __shared__ uint32_t s_mask[2 * kPreBlock];
    __shared__ uint32_t s_wsum[kPreBlock / 64], s_part[2 * (kPreBlock / 64)];
    const int64_t slot0 = (int64_t)blockIdx.x * kPreBlock;
    // With table_out, the frame's one item comes as an argument: workgroup 0
    // writes it to the table the later stages read and zeroes the frame
    // counts (which k_totals adds to after this kernel), so no launch of its
    // own precedes the frame.
    if (table_out && blockIdx.x == 0) {
        static_assert(sizeof(Item) % 4 == 0, "item words");
        const uint32_t* src = reinterpret_cast<const uint32_t*>(&item0);
        uint32_t* dst = reinterpret_cast<uint32_t*>(table_out);
        for (int k = threadIdx.x; k < (int)(sizeof(Item) / 4); k += kPreBlock) dst[k] = src[k];
        if (threadIdx.x < 2) totals[threadIdx.x] = 0u;
    }
    Item it;
    if (table_out)
        it = item0;
    else
        it = items[dims.n_items == 1 ? 0 : item_of_slot(items, dims.n_items, slot0)];
    const ss_camera cam = it.cam;
    const Inputs in{it.means, it.scales, it.quats, it.opacity, it.sh, it.sh_degree, it.sh_stride};
    const int64_t n = it.n;
    const int tx_n = it.tx_n, ty_n = it.ty_n, by0 = it.by0, by1 = it.by1;
    const int64_t first = slot0 - it.g_off;       // local index of this block's first lane
    const int64_t i = first + threadIdx.x;        // Gaussian of the item
    const int64_t o = slot0 + threadIdx.x;        // its record slot
    const bool real = i < n && o < dims.n_slots;

    float m0 = 0.f, m1 = 0.f, m2 = 1.f, s0 = 0.f, s1 = 0.f, s2 = 0.f, op = 0.f;
    float4 qr = make_float4(0.f, 0.f, 0.f, 0.f);
    if (real) {
        m0 = in.means[3 * i]; m1 = in.means[3 * i + 1]; m2 = in.means[3 * i + 2];
        s0 = in.scales[3 * i]; s1 = in.scales[3 * i + 1]; s2 = in.scales[3 * i + 2];
        qr = *reinterpret_cast<const float4*>(in.quats + 4 * i);
        op = in.opacity[i];
    }

    // The record, its count and its tile set; 0 for a padding slot or a culled
    // Gaussian (whose record is zeroed), and for an AccuTile record, whose
    // count and tile set the wave computes afterwards (defer).
    float4 g4 = make_float4(0.f, 0.f, 0.f, 0.f), q4 = g4;
    bool defer = false;
    auto record = [&]() -> uint32_t {
        const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
        if (i >= n) {  // padding slot between items
            geom[kRec * o] = zero; conic[kRec * o] = zero; counts[o] = 0u;
            dkeys[o] = kCulledKey;
            tsets[o] = make_uint4(0u, 0u, 0u, 0u);
            return 0u;
        }

        bool ok = finite_f(m0) && finite_f(m1) && finite_f(m2) && finite_f(s0) && finite_f(s1) &&
                  finite_f(s2) && finite_f(qr.x) && finite_f(qr.y) && finite_f(qr.z) &&
                  finite_f(qr.w) && finite_f(op) && (op > 0.0f);

        // camera space p_c = R mu + t
        const double R0 = cam.R[0], R1 = cam.R[1], R2 = cam.R[2], R3 = cam.R[3], R4 = cam.R[4],
                     R5 = cam.R[5], R6 = cam.R[6], R7 = cam.R[7], R8 = cam.R[8];
        const double mx = m0, my = m1, mz = m2;
        const double x = ((R0 * mx + R1 * my) + R2 * mz) + (double)cam.t[0];
        const double y = ((R3 * mx + R4 * my) + R5 * mz) + (double)cam.t[1];
        const double z = ((R6 * mx + R7 * my) + R8 * mz) + (double)cam.t[2];
        ok = ok && (z > (double)cam.near_z);

        // quaternion (w, x, y, z) normalised in FP64
        double qw = qr.x, qx = qr.y, qy = qr.z, qz = qr.w;
        const double nn = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
        ok = ok && (nn > 0.0);
        if (!ok) {
            geom[kRec * o] = zero; conic[kRec * o] = zero; counts[o] = 0u;
            dkeys[o] = kCulledKey;
            tsets[o] = make_uint4(0u, 0u, 0u, 0u);
            return 0u;
        }
        const double fx = cam.fx, fy = cam.fy;
        const double u = (fx * x) / z + (double)cam.cx;
        const double v = (fy * y) / z + (double)cam.cy;

        const double qn = sqrt(nn);
        qw = qw / qn; qx = qx / qn; qy = qy / qn; qz = qz / qn;
        double Rq[9];
        Rq[0] = 1.0 - 2.0 * (qy * qy + qz * qz);
        Rq[1] = 2.0 * (qx * qy - qw * qz);
        Rq[2] = 2.0 * (qx * qz + qw * qy);
        Rq[3] = 2.0 * (qx * qy + qw * qz);
        Rq[4] = 1.0 - 2.0 * (qx * qx + qz * qz);
        Rq[5] = 2.0 * (qy * qz - qw * qx);
        Rq[6] = 2.0 * (qx * qz - qw * qy);
        Rq[7] = 2.0 * (qy * qz + qw * qx);
        Rq[8] = 1.0 - 2.0 * (qx * qx + qy * qy);

        // Sigma_3D = (R S)(R S)^T
        const double sc[3] = {(double)s0, (double)s1, (double)s2};
        double M[9];
    #pragma unroll
        for (int r = 0; r < 3; ++r)
    #pragma unroll
            for (int c = 0; c < 3; ++c) M[3 * r + c] = Rq[3 * r + c] * sc[c];
        double S3[9];
    #pragma unroll
        for (int r = 0; r < 3; ++r)
    #pragma unroll
            for (int c = 0; c < 3; ++c)
                S3[3 * r + c] = (M[3 * r] * M[3 * c] + M[3 * r + 1] * M[3 * c + 1]) +
                                M[3 * r + 2] * M[3 * c + 2];

        // EWA projection with the Jacobian at the FOV-clamped mean
        const double limx = kFovClamp * ((0.5 * (double)cam.width) / fx);
        const double limy = kFovClamp * ((0.5 * (double)cam.height) / fy);
        double txz = x / z, tyz = y / z;
        txz = txz < -limx ? -limx : txz;
        txz = txz > limx ? limx : txz;
        tyz = tyz < -limy ? -limy : tyz;
        tyz = tyz > limy ? limy : tyz;
        const double J00 = fx / z, J02 = -(fx * txz) / z;
        const double J11 = fy / z, J12 = -(fy * tyz) / z;
        const double Rc[9] = {R0, R1, R2, R3, R4, R5, R6, R7, R8};
        double T[6];
    #pragma unroll
        for (int j = 0; j < 3; ++j) {
            T[j] = J00 * Rc[j] + J02 * Rc[6 + j];
            T[3 + j] = J11 * Rc[3 + j] + J12 * Rc[6 + j];
        }
        double V[6];
    #pragma unroll
        for (int r = 0; r < 2; ++r)
    #pragma unroll
            for (int c = 0; c < 3; ++c)
                V[3 * r + c] = (T[3 * r] * S3[c] + T[3 * r + 1] * S3[3 + c]) + T[3 * r + 2] * S3[6 + c];
        const double s00 = (V[0] * T[0] + V[1] * T[1]) + V[2] * T[2];
        const double s01 = (V[0] * T[3] + V[1] * T[4]) + V[2] * T[5];
        const double s11 = (V[3] * T[3] + V[4] * T[4]) + V[5] * T[5];
        const double A = s00 + kDilation, B = s01, C = s11 + kDilation;
        const double D = A * C - B * B;
        const float ca = (float)(C / D), cb = (float)(-B / D), cc = (float)(A / D);
        const float tt = (float)(2.0 * log(255.0 * (double)op));
        if (!(D > 0.0) || (mode != SS_TILE_3SIGMA && !(tt > 0.0f))) {
            geom[kRec * o] = zero; conic[kRec * o] = zero; counts[o] = 0u;
            dkeys[o] = kCulledKey;
            tsets[o] = make_uint4(0u, 0u, 0u, 0u);
            return 0u;
        }

        g4 = make_float4((float)u, (float)v, (float)z, tt);
        q4 = make_float4(ca, cb, cc, op);
        geom[kRec * o] = g4;
        conic[kRec * o] = q4;
        if (mode == SS_TILE_ACCUTILE) {   // tile set computed by the wave below
            defer = true;
            return 0u;
        }
        uint64_t mask;
        uint32_t origin;
        const uint32_t cnt = rect_tile_set(g4, q4, mode, tx_n, ty_n, by0, by1, &mask, &origin);
        tsets[o] = make_uint4((uint32_t)mask, (uint32_t)(mask >> 32), origin, cnt);
        counts[o] = cnt;
        dkeys[o] = cnt ? __float_as_uint(g4.z) : kCulledKey;
        return cnt;
    };
    uint32_t cnt = o < dims.n_slots ? record() : 0u;

    if (mode == SS_TILE_ACCUTILE) {   // workgroup-uniform
        uint64_t mask;
        uint32_t origin;
        const uint32_t c = accutile_tile_set_wg(defer, g4, q4, tx_n, ty_n, by0, by1, s_rec, s_incl,
                                                s_nb, s_cnt, s_mask, s_wsum, &mask, &origin);
        if (defer) {
            cnt = c;
            tsets[o] = make_uint4((uint32_t)mask, (uint32_t)(mask >> 32), origin, cnt);
            counts[o] = cnt;
            dkeys[o] = cnt ? __float_as_uint(g4.z) : kCulledKey;
        }
    }

    // This workgroup's share of the pair count P and of the Gaussians with
    // tiles, summed by k_totals: plain stores, since thousands of atomics on
    // one address would serialise.
    uint32_t sp = cnt, sv = cnt ? 1u : 0u;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        sp += __shfl_xor(sp, d, 64);
        sv += __shfl_xor(sv, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        s_part[2 * (threadIdx.x >> 6)] = sp;
        s_part[2 * (threadIdx.x >> 6) + 1] = sv;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t p = 0, v = 0;
        for (int k = 0; k < kPreBlock / 64; ++k) {
            p += s_part[2 * k];
            v += s_part[2 * k + 1];
        }
        partials[2 * blockIdx.x] = p;
        partials[2 * blockIdx.x + 1] = v;
    }
}

// Real SH basis up to `degree` at the unit direction from the camera centre
// (-R^T t) to the mean (Sec. 3.2.1; the standard 3DGS constants).
__device__ __forceinline__ void sh_basis(const ss_camera& cam, float m0, float m1, float m2,
                                         int degree, float Y[16]) {
    const float cpx = -((cam.R[0] * cam.t[0] + cam.R[3] * cam.t[1]) + cam.R[6] * cam.t[2]);
    const float cpy = -((cam.R[1] * cam.t[0] + cam.R[4] * cam.t[1]) + cam.R[7] * cam.t[2]);
    const float cpz = -((cam.R[2] * cam.t[0] + cam.R[5] * cam.t[1]) + cam.R[8] * cam.t[2]);
    float dx = m0 - cpx, dy = m1 - cpy, dz = m2 - cpz;
    const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
    dx *= inv; dy *= inv; dz *= inv;
    Y[0] = kSH0;
    if (degree >= 1) {
        Y[1] = -kSH1 * dy; Y[2] = kSH1 * dz; Y[3] = -kSH1 * dx;
    }
    if (degree >= 2) {
        const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
        Y[4] = kSH2a * (dx * dy);
        Y[5] = -kSH2a * (dy * dz);
        Y[6] = kSH2b * (2.0f * zz - xx - yy);
        Y[7] = -kSH2a * (dx * dz);
        Y[8] = kSH2c * (xx - yy);
        if (degree >= 3) {
            Y[9] = -kSH3a * dy * (3.0f * xx - yy);
            Y[10] = kSH3b * (dx * dy * dz);
            Y[11] = -kSH3c * dy * (4.0f * zz - xx - yy);
            Y[12] = kSH3d * dz * (2.0f * zz - 3.0f * xx - 3.0f * yy);
            Y[13] = -kSH3c * dx * (4.0f * zz - xx - yy);
            Y[14] = kSH3e * dz * (xx - yy);
            Y[15] = -kSH3a * dx * (xx - 3.0f * yy);
        }
    }
}

__device__ __forceinline__ float4 colour_of(float cr, float cg, float cb) {
    return make_float4(fmaxf(cr + 0.5f, 0.0f), fmaxf(cg + 0.5f, 0.0f), fmaxf(cb + 0.5f, 0.0f),
                       0.0f);
}

// View-dependent colour from SH (FP32), for the Gaussians with tiles (the
// others get rgb = 0), when every SH row starts 16-byte aligned (a row of a
// multiple of 4 floats from an aligned base).  The wave lists its lanes with
// tiles, then copies their rows to LDS kColRows at a time with 16-byte loads,
// consecutive lanes on consecutive pieces of a row (a row's 1.5 cache lines
// read by one instruction, rows of Gaussians without tiles not read), and
// each listed lane reads its own row back.  A lane loading a whole row by
// itself would make every load instruction touch 64 cache lines.
constexpr int kColRows = 32;               // rows staged per round
constexpr int kColPitch = 13;              // 16-byte pieces per staged row: 12 + 1 (banks)
__device__ __forceinline__ void colour_rows_block(const Item* __restrict__ items,
                                                  const BatchDims& dims,
                                                  const uint32_t* __restrict__ counts,
                                                  float4* __restrict__ rgb_out, int64_t slot0,
                                                  float4* __restrict__ s_rows,
                                                  uint32_t* __restrict__ s_lane) {
    const Item& it = items[dims.n_items == 1 ? 0 : item_of_slot(items, dims.n_items, slot0)];
    const int lane = (int)threadIdx.x;
    const int64_t first = slot0 - it.g_off;
    const int64_t i = first + lane;
    const int64_t o = slot0 + lane;
    const bool vis = o < dims.n_slots && i < it.n && counts[o] != 0u;
    const uint64_t vm = __ballot(vis);
    const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(vm >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)vm, 0u));
    if (vis) s_lane[rank] = (uint32_t)lane;
    __syncthreads();
    const int n_vis = __popcll(vm);
    const int nb = (it.sh_degree + 1) * (it.sh_degree + 1);
    const int q = (3 * nb + 3) / 4;                   // 16-byte pieces holding the nb coefficients
    const uint32_t urow4 = (uint32_t)(3 * it.sh_stride) / 4u;
    const float4* base = reinterpret_cast<const float4*>(it.sh + first * (3 * (int64_t)it.sh_stride));
    float Y[16];
    if (vis)
        sh_basis(it.cam, ld_global(it.means + 3 * i), ld_global(it.means + 3 * i + 1),
                 ld_global(it.means + 3 * i + 2), it.sh_degree, Y);
    float4 col = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int r0 = 0; r0 < n_vis; r0 += kColRows) {
        const int rows = n_vis - r0 < kColRows ? n_vis - r0 : kColRows;
        const int pieces = rows * q;
        // all loads of the round are issued before the first LDS store
        constexpr int kPer = kColRows * 12 / kBlock;
        float4 v[kPer];
        int dst[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int p = u * kBlock + lane;
            const bool ok = p < pieces;
            const int r = ok ? p / q : 0, j = ok ? p - r * q : 0;
            dst[u] = ok ? r * kColPitch + j : -1;
            const uint32_t L = s_lane[r0 + r];          // r0 + r < n_vis
            v[u] = ok ? ld_global(base + (uint64_t)L * urow4 + j) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u)
            if (dst[u] >= 0) s_rows[dst[u]] = v[u];
        __syncthreads();
        if (vis && (int)rank >= r0 && (int)rank < r0 + kColRows) {
            const float4* row = s_rows + ((int)rank - r0) * kColPitch;
            float h[48];
#pragma unroll
            for (int j = 0; j < 12; ++j) {
                const float4 x = j < q ? row[j] : make_float4(0.f, 0.f, 0.f, 0.f);
                h[4 * j] = x.x; h[4 * j + 1] = x.y; h[4 * j + 2] = x.z; h[4 * j + 3] = x.w;
            }
            float cr = 0.f, cg = 0.f, cbl = 0.f;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                if (k < nb) {
                    cr = fmaf(Y[k], h[3 * k], cr);
                    cg = fmaf(Y[k], h[3 * k + 1], cg);
                    cbl = fmaf(Y[k], h[3 * k + 2], cbl);
                }
            }
            col = colour_of(cr, cg, cbl);
        }
        __syncthreads();
    }
    if (o < dims.n_slots) rgb_out[o] = col;
}

// Workgroup b colours the slots of blocks b, b + grid, ...: one block each
// when the grid covers the slots, fewer workgroups when the kernel runs beside
// the stages that follow the geometry kernel.
__global__ __launch_bounds__(kBlock) void k_colour_rows(const Item* __restrict__ items,
                                                        BatchDims dims,
                                                        const uint32_t* __restrict__ counts,
                                                        float4* __restrict__ rgb_out) {
    __shared__ float4 s_rows[kColRows * kColPitch];
    __shared__ uint32_t s_lane[kBlock];
    const int64_t blocks = (dims.n_slots + kBlock - 1) / kBlock;
    for (int64_t b = blockIdx.x; b < blocks; b += gridDim.x) {
        colour_rows_block(items, dims, counts, rgb_out, b * kBlock, s_rows, s_lane);
        __syncthreads();              // the next block rewrites s_lane and s_rows
    }
}

// The same for any row layout: one wave per workgroup stages the SH rows of
// its visible Gaussians through LDS with coalesced loads.
__global__ __launch_bounds__(kBlock) void k_colour(const Item* __restrict__ items, BatchDims dims,
                                                   const uint32_t* __restrict__ counts,
                                                   float4* __restrict__ rgb_out) {
    __shared__ float s_sh[kBlock * kShPitch];
    __shared__ uint32_t s_vis[kBlock];
    const int64_t slot0 = (int64_t)blockIdx.x * kBlock;
    const Item& it = items[dims.n_items == 1 ? 0 : item_of_slot(items, dims.n_items, slot0)];
    const int64_t n = it.n;
    const int64_t first = slot0 - it.g_off;
    const int64_t i = first + threadIdx.x;
    const int64_t o = slot0 + threadIdx.x;
    const bool vis = i < n && o < dims.n_slots && counts[o] > 0u;
    s_vis[threadIdx.x] = vis ? 1u : 0u;
    const int nb = (it.sh_degree + 1) * (it.sh_degree + 1);
    __syncthreads();
    if (first < n) stage_sh(it.sh, first, n, 3 * it.sh_stride, 3 * nb, s_vis, s_sh);
    __syncthreads();
    if (o >= dims.n_slots) return;
    if (!vis) {
        rgb_out[o] = make_float4(0.f, 0.f, 0.f, 0.f);
        return;
    }
    float Y[16];
    sh_basis(it.cam, ld_global(it.means + 3 * i), ld_global(it.means + 3 * i + 1),
             ld_global(it.means + 3 * i + 2), it.sh_degree, Y);
    const float* h = s_sh + threadIdx.x * kShPitch;
    float cr = 0.f, cg = 0.f, cbl = 0.f;
    for (int k = 0; k < nb; ++k) {
        cr = fmaf(Y[k], h[3 * k], cr);
        cg = fmaf(Y[k], h[3 * k + 1], cg);
        cbl = fmaf(Y[k], h[3 * k + 2], cbl);
    }
    rgb_out[o] = colour_of(cr, cg, cbl);
}

// totals += (sum of the pair-count partials, sum of the visible-count
// partials) over nb workgroups of k_preprocess: each workgroup sums a
// contiguous run of partials and adds its two sums with one atomic each
// (a few dozen atomics on one address; the totals were zeroed by
// k_write_items or, for a frame of one item, by k_preprocess).
__global__ __launch_bounds__(1024) void k_totals(const uint32_t* __restrict__ partials, int64_t nb,
                                                 uint64_t* __restrict__ totals) {
    __shared__ uint64_t s_p[16], s_v[16];
    uint64_t p = 0, v = 0;
    const int64_t per = (nb + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < nb ? lo + per : nb;
    // (P, visible) pairs as 8-byte loads
    const uint2* __restrict__ pv = reinterpret_cast<const uint2*>(partials);
    for (int64_t b = lo + threadIdx.x; b < hi; b += 1024) {
        const uint2 x = pv[b];
        p += x.x;
        v += x.y;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        p += __shfl_xor(p, d, 64);
        v += __shfl_xor(v, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        s_p[threadIdx.x >> 6] = p;
        s_v[threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t tp = 0, tv = 0;
        for (int w = 0; w < 16; ++w) {
            tp += s_p[w];
            tv += s_v[w];
        }
        if (tp) atomicAdd((unsigned long long*)&totals[0], (unsigned long long)tp);
        if (tv) atomicAdd((unsigned long long*)&totals[1], (unsigned long long)tv);
    }
}

}  // namespace

namespace {
// Waves per CU of the colour kernel when it runs beside the depth order, scan,
// emit and sort (measured: 2, 4 and 8 per CU; a full grid slowed those stages
// by more than it saved).
constexpr int kColourSideWaves = 8;

// Compute units of the current device (cached per device).
int compute_units() {
    static int cached[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            return 256;
        cached[dev] = cus;
    }
    return cached[dev];
}
}  // namespace

hipError_t launch_preprocess(const Item* items, const BatchDims& d, int mode, const ss_frame& f,
                             bool sh_rows16, hipStream_t s, const SideStream* side,
                             const Item* host_single, Item* table) {
    // per-workgroup partial counts go to the emit stage's scratch, free until then
    const int64_t pgrid = (d.n_slots + kPreBlock - 1) / kPreBlock;
    const int64_t grid = (d.n_slots + kBlock - 1) / kBlock;       // the colour kernels'
    if (host_single && grid == 0) {
        // no geometry kernel to carry the item: the table still needs it
        const hipError_t e = write_items(table, host_single, 1, s, f.totals);
        if (e != hipSuccess) return e;
        host_single = nullptr;
    }
    if (grid > 0) {
        const Item item0 = host_single ? *host_single : Item{};
        hipLaunchKernelGGL(k_preprocess, dim3((unsigned)pgrid), dim3(kPreBlock), 0, s, items, d,
                           mode, reinterpret_cast<float4*>(f.geom),
                           reinterpret_cast<float4*>(f.conic), f.counts, f.depth_keys,
                           reinterpret_cast<uint4*>(f.tile_sets), f.emit_tmp, item0,
                           host_single ? table : nullptr, f.totals);
        // the colour needs the counts; only the blend needs the colour
        hipStream_t cs = s;
        if (side) {
            hipError_t e = hipEventRecord(side->fork, s);
            if (e == hipSuccess) e = hipStreamWaitEvent(side->stream, side->fork, 0);
            if (e != hipSuccess) return e;
            cs = side->stream;
        }
        // beside the later stages the colour kernel takes a few waves per CU,
        // leaving the CUs to their latency-bound kernels
        unsigned cgrid = (unsigned)grid;
        if (side && sh_rows16) {
            const int64_t cap = (int64_t)kColourSideWaves * compute_units();
            cgrid = (unsigned)(grid < cap ? grid : cap);
        }
        hipLaunchKernelGGL(sh_rows16 ? k_colour_rows : k_colour, dim3(cgrid), dim3(kBlock), 0, cs,
                           items, d, f.counts, reinterpret_cast<float4*>(f.rgb));
        if (side) {
            const hipError_t e = hipEventRecord(side->join, side->stream);
            if (e != hipSuccess) return e;
        }
    } else if (side) {
        const hipError_t e = hipEventRecord(side->join, s);     // nothing to wait for
        if (e != hipSuccess) return e;
    }
    if (pgrid > 0) {
        // about 1024 partials per reducing workgroup
        const int64_t tg = (pgrid + 1023) / 1024 < 64 ? (pgrid + 1023) / 1024 : 64;
        hipLaunchKernelGGL(k_totals, dim3((unsigned)tg), dim3(1024), 0, s, f.emit_tmp, pgrid,
                           f.totals);
    }
    return hipGetLastError();
}

// Writes items [first, first + count) of the table; with totals, also zeroes
// the frame counts the preprocess stage accumulates.
__global__ void k_write_items(Item* __restrict__ table, ItemPack pack, int first, int count,
                              uint64_t* __restrict__ totals) {
    const int k = threadIdx.x;
    if (k < count) table[first + k] = pack.it[k];
    if (totals && k < 2) totals[k] = 0u;
}

hipError_t write_items(Item* table, const Item* host_items, int n_items, hipStream_t s,
                       uint64_t* totals) {
    for (int first = 0; first < n_items; first += kPack) {
        ItemPack pack;
        const int count = n_items - first < kPack ? n_items - first : kPack;
        for (int k = 0; k < count; ++k) pack.it[k] = host_items[first + k];
        hipLaunchKernelGGL(k_write_items, dim3(1), dim3(kPack), 0, s, table, pack, first, count,
                           first == 0 ? totals : nullptr);
    }
    return hipGetLastError();
}

}  // namespace ss

// Internal declarations of the gfx950 Speedy-Splat library.
//
// Build flags (see build.py): -O3 --offload-arch=gfx950 -ffp-contract=off and
// packed FP32 disabled.  With contraction off every + - * / sqrt below is one
// IEEE operation rounded once, in the written order; FP64 division and square
// root are correctly rounded on gfx950, so the FP64 geometry is reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/speedysplat.h"

namespace ss {

constexpr int kTile = 16;                 // Sec. 3.2: 16 x 16 pixel tiles
constexpr double kDilation = 0.3;         // added to the diagonal of Sigma_2D
constexpr double kFovClamp = 1.3;         // J evaluated with x/z, y/z clamped to 1.3x half-FOV
constexpr double kDiscFloor = 0.1;        // floor of the eigenvalue discriminant (3-sigma)
constexpr float kAlphaMax = 0.99f;        // upper clamp of alpha
constexpr float kTMin = 1e-4f;            // transmittance stop
constexpr float kAlphaMin = 1.0f / 255.0f;  // inclusion cutoff, used as q <= t
constexpr uint32_t kCulledKey = 0xffffffffu;  // depth-order key of a slot with no tiles
// A Gaussian's record is geom (u, v, depth, t) followed by conic (a, b, c,
// sigma): float4s kRec * i and kRec * i + 1 of frame.geom (frame.conic is
// frame.geom + 4 floats), so a gather of both touches one 32-byte piece.
constexpr int kRec = 2;

// ---------------------------------------------------------------- tile geometry
//
// All tile decisions are FP64 functions of the stored FP32 record
// (u, v, t) = geom.xyw and (a, b, c) = conic.xyz.

struct Ellipse {
    double u, v, a, b, c, t, det, hx, hy;
    int x0, x1, y0, y1;  // inclusive tile rectangle (rows clipped to the frame's band)
    bool cols;           // AccuTile walks columns (decided on the image's rectangle)
};

// Edge -> tile index: divide by the tile size, round down, clip to the grid.
__device__ __forceinline__ int tile_lo(double x, int n) {
    double f = floor(x / 16.0);
    f = f < 0.0 ? 0.0 : f;
    f = f > (double)n ? (double)n : f;
    return (int)f;
}
__device__ __forceinline__ int tile_hi(double x, int n) {
    double f = floor(x / 16.0);
    f = f < -1.0 ? -1.0 : f;
    f = f > (double)(n - 1) ? (double)(n - 1) : f;
    return (int)f;
}

// Sets up the record ellipse and the mode's tile rectangle, then clips its rows
// to the frame's band of tile rows [by0, by1) (the whole image: 0, ty_n).
// AccuTile's walking direction is decided on the rectangle within the image,
// before the band clip, so a band's tiles are exactly the image's tiles in
// those rows.  False when the record cannot touch a tile of the band (culled
// record, or rectangle outside the image or the band).
__device__ __forceinline__ bool ellipse_setup(float4 g, float4 q, int mode, int tx_n, int ty_n,
                                              int by0, int by1, Ellipse& e) {
    e.u = g.x; e.v = g.y; e.t = g.w;
    e.a = q.x; e.b = q.y; e.c = q.z;
    e.det = e.a * e.c - e.b * e.b;
    e.hx = 0.0; e.hy = 0.0;
    if (!(e.det > 0.0)) return false;
    double xl, xh, yl, yh;
    if (mode == SS_TILE_3SIGMA) {
        // Eq. radius: r = ceil(3 sqrt(lambda_max)) of the record covariance.
        double sxx = e.c / e.det, syy = e.a / e.det;
        double mid = 0.5 * (sxx + syy);
        double disc = mid * mid - 1.0 / e.det;
        disc = disc < kDiscFloor ? kDiscFloor : disc;
        double lam = mid + sqrt(disc);
        double r = ceil(3.0 * sqrt(lam));
        xl = e.u - r; xh = e.u + r; yl = e.v - r; yh = e.v + r;
    } else {
        if (!(e.t > 0.0)) return false;
        // SnugBox (Sec. 4.1.1): extremes of a x^2 + 2bxy + c y^2 = t.
        e.hx = sqrt((e.t * e.c) / e.det);
        e.hy = sqrt((e.t * e.a) / e.det);
        xl = e.u - e.hx; xh = e.u + e.hx; yl = e.v - e.hy; yh = e.v + e.hy;
    }
    e.x0 = tile_lo(xl, tx_n); e.x1 = tile_hi(xh, tx_n);
    e.y0 = tile_lo(yl, ty_n); e.y1 = tile_hi(yh, ty_n);
    e.cols = mode == SS_TILE_ACCUTILE && (e.y1 - e.y0 > e.x1 - e.x0);
    // A row band k of a clipped rectangle is evaluated exactly as in the whole
    // image: its lower boundary is 16 (y0 + k) whether or not it is the first
    // (16 y0 lies in [box bottom, box top] for every row but the rectangle's
    // first), so clipping y0 changes no span.
    e.y0 = e.y0 < by0 ? by0 : e.y0;
    e.y1 = e.y1 > by1 - 1 ? by1 - 1 : e.y1;
    return e.x0 <= e.x1 && e.y0 <= e.y1;
}

// Intersections of the ellipse with the horizontal line y = Y (x roots).
__device__ __forceinline__ void row_roots(const Ellipse& e, double Y, double& xl, double& xr) {
    double dy = Y - e.v;
    double rad = e.t * e.a - (e.det * dy) * dy;
    double s = sqrt(rad > 0.0 ? rad : 0.0);
    double bd = e.b * dy;
    xl = e.u + (-bd - s) / e.a;
    xr = e.u + (-bd + s) / e.a;
}

// Intersections with the vertical line x = X (Eq. ellipse_intersect, y roots).
__device__ __forceinline__ void col_roots(const Ellipse& e, double X, double& yt, double& yb) {
    double dx = X - e.u;
    double rad = e.t * e.c - (e.det * dx) * dx;
    double s = sqrt(rad > 0.0 ? rad : 0.0);
    double bd = e.b * dx;
    yt = e.v + (-bd - s) / e.c;
    yb = e.v + (-bd + s) / e.c;
}

// AccuTile (Alg. 1) walks a record's tile rectangle in bands, rows of tiles
// (or columns, when the rectangle has more rows than columns).  A band's
// extent along the other axis is the SnugBox extremal point when that lies
// inside the band, else the extreme of the ellipse's intersections with the
// two band boundaries.  accutile_band evaluates band k (0-based, major index
// y0 + k or x0 + k) on its own; its lower boundary is the upper boundary of
// band k - 1, min(16 (y0 + k), box top), computed with the same FP64
// operations, so evaluating the bands independently or in order gives the
// same spans.  False when the band's span is empty.
__device__ __forceinline__ bool accutile_band(const Ellipse& e, bool cols, int k, int tx_n,
                                              int ty_n, int& lo, int& hi) {
    if (!cols) {
        const int ty = e.y0 + k;
        const double kk = (e.b / e.c) * e.hx;
        const double y_left = e.v + kk, y_right = e.v - kk;
        const double box_b = e.v - e.hy, box_t = e.v + e.hy;
        const double x_min = e.u - e.hx, x_max = e.u + e.hx;
        double ylo;
        if (k == 0) {
            ylo = 16.0 * e.y0;
            ylo = ylo < box_b ? box_b : ylo;
        } else {
            ylo = 16.0 * ty;
            ylo = ylo > box_t ? box_t : ylo;
        }
        double yhi = 16.0 * ty + 16.0;
        yhi = yhi > box_t ? box_t : yhi;
        double l0, r0, l1, r1;
        row_roots(e, ylo, l0, r0);
        row_roots(e, yhi, l1, r1);
        const double left = (ylo <= y_left && y_left <= yhi) ? x_min : (l0 < l1 ? l0 : l1);
        const double right = (ylo <= y_right && y_right <= yhi) ? x_max : (r0 > r1 ? r0 : r1);
        lo = tile_lo(left, tx_n);
        hi = tile_hi(right, tx_n);
        lo = lo < e.x0 ? e.x0 : lo;
        hi = hi > e.x1 ? e.x1 : hi;
        return lo <= hi;
    }
    const int tx = e.x0 + k;
    const double m = (e.b / e.a) * e.hy;
    const double x_top = e.u + m, x_bot = e.u - m;
    const double box_l = e.u - e.hx, box_r = e.u + e.hx;
    const double y_min = e.v - e.hy, y_max = e.v + e.hy;
    double xlo;
    if (k == 0) {
        xlo = 16.0 * e.x0;
        xlo = xlo < box_l ? box_l : xlo;
    } else {
        xlo = 16.0 * tx;
        xlo = xlo > box_r ? box_r : xlo;
    }
    double xhi = 16.0 * tx + 16.0;
    xhi = xhi > box_r ? box_r : xhi;
    double t0, b0, t1, b1;
    col_roots(e, xlo, t0, b0);
    col_roots(e, xhi, t1, b1);
    const double top = (xlo <= x_top && x_top <= xhi) ? y_min : (t0 < t1 ? t0 : t1);
    const double bot = (xlo <= x_bot && x_bot <= xhi) ? y_max : (b0 > b1 ? b0 : b1);
    lo = tile_lo(top, ty_n);
    hi = tile_hi(bot, ty_n);
    lo = lo < e.y0 ? e.y0 : lo;
    hi = hi > e.y1 ? e.y1 : hi;
    return lo <= hi;
}

// AccuTile walks columns when the tile extent within the image has more rows
// than columns.
__device__ __forceinline__ bool span_columns(const Ellipse& e, int mode) {
    return mode == SS_TILE_ACCUTILE && e.cols;
}

// Side of the tile window a tile set records: a record whose tile rectangle
// fits kSetSide x kSetSide tiles stores its tiles as a bit mask over that
// window, bit r * kSetSide + c for tile (x0 + c, y0 + r).
constexpr int kSetSide = 8;

// 3-sigma / SnugBox tile set: the whole rectangle.  Returns the tile count
// and, when the rectangle fits the window, sets *mask (its row run repeated
// once per row) and *origin = x0 | y0 << 16; otherwise *mask = 0 (the emit
// stage re-walks the rows).
__device__ __forceinline__ uint32_t rect_tile_set(float4 g, float4 q, int mode, int tx_n,
                                                  int ty_n, int by0, int by1, uint64_t* mask,
                                                  uint32_t* origin) {
    *mask = 0ull;
    *origin = 0u;
    Ellipse e;
    if (!ellipse_setup(g, q, mode, tx_n, ty_n, by0, by1, e)) return 0u;
    const uint32_t w = (uint32_t)(e.x1 - e.x0 + 1), h = (uint32_t)(e.y1 - e.y0 + 1);
    if (w <= (uint32_t)kSetSide && h <= (uint32_t)kSetSide) {
        *mask = ((1ull << w) - 1ull) * (0x0101010101010101ull >> (8u * (kSetSide - h)));
        *origin = (uint32_t)e.x0 | ((uint32_t)(e.y0 - by0) << 16);
    }
    return w * h;
}

// Workgroups are dispatched round-robin over the 8 XCDs of MI355X.  This maps
// launch index b (grid = 8 * ceil(n/8)) to item b % 8 * ceil(n/8) + b / 8, so
// every XCD walks a contiguous run of items and keeps their shared data in its
// own L2.  Returns -1 for the padding indices.
__device__ __forceinline__ int xcd_contiguous(int b, int n) {
    int per = (n + 7) >> 3;
    int t = (b & 7) * per + (b >> 3);
    return t < n ? t : -1;
}

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

// ---------------------------------------------------------------- frame counts
//
// The stages after the preprocess can run without the host reading the frame
// counts back: launched over host bounds (the record slots, the pair
// workspace's capacity), they read the counts the preprocess stage left in
// device memory (ss_frame.totals: word 0 the pair count P, word 1 the
// Gaussians with tiles).  A count above its bound (a pair workspace too
// small for the frame) reads as 0, so nothing is written past the buffers.
// totals == nullptr: the bound is the count (the host read it back).
__device__ __forceinline__ uint64_t frame_count(const uint64_t* totals, int word,
                                                uint64_t bound) {
    if (!totals) return bound;
    const uint64_t v = totals[word];
    return v <= bound ? v : 0u;
}

// ---------------------------------------------------------------- render items
//
// Every launch renders a batch of one or more items (a camera, a resident
// scene and an output image).  Per-Gaussian buffers hold each item's records
// in a run of "slots" starting at g_off (a multiple of 256, so a 256-lane
// workgroup never spans two items); tiles carry a global id tile_off + local
// id; per-pixel buffers hold each item's pixels from pix_off.  A single frame
// is the batch of one item with g_off = tile_off = pix_off = 0.  The item
// table lives in device memory (written by write_items).

constexpr int kSlotAlign = 256;

struct Item {
    ss_camera cam;
    const float* means;
    const float* scales;
    const float* quats;
    const float* opacity;
    const float* sh;
    float* out_rgb;       // [3, H, W]
    int64_t n;            // Gaussians of the scene
    int64_t g_off;        // first record slot
    int64_t pix_off;      // first pixel in the per-pixel buffers
    int32_t sh_degree, sh_stride;
    int32_t tx_n, ty_n;   // tile grid of the item's image
    int32_t tile_off;     // first global tile id
    int32_t by0, by1;     // the item's band of tile rows [by0, by1) (the image: 0, ty_n);
                          // its tiles, pixels and image cover these rows only
    int32_t pad_;
};

// Loads through pointers read from an item table.  The compiler cannot tell
// that such a pointer is global and would emit flat loads, whose completion
// is counted together with LDS and scalar loads, so that every LDS wait also
// waits for them; these take the global path explicitly.
typedef float ss_v4f __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) float ss_gfloat;
typedef const __attribute__((address_space(1))) ss_v4f ss_gv4f;

__device__ __forceinline__ float ld_global(const float* p) { return *(ss_gfloat*)p; }

__device__ __forceinline__ float4 ld_global(const float4* p) {
    const ss_v4f v = *(ss_gv4f*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}

// The item table buffer holds the n_items items, then (from the next 256-byte
// boundary) the blend's tile work order, one u32 per tile, then (from the next
// 256-byte boundary) the 8 per-XCD work counters of the persistent blend.
inline int64_t table_bytes(int n_items, int n_tiles) {
    const int64_t items = ((int64_t)sizeof(Item) * n_items + 255) / 256 * 256;
    return items + ((int64_t)n_tiles * 4 + 255) / 256 * 256 + 256;
}
inline uint32_t* tile_order_of(void* table, int n_items) {
    return reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(table) +
                                       ((int64_t)sizeof(Item) * n_items + 255) / 256 * 256);
}
inline uint32_t* tile_queue_of(void* table, int n_items, int n_tiles) {
    return tile_order_of(table, n_items) + ((int64_t)n_tiles * 4 + 255) / 256 * 64;
}

struct BatchDims {
    int32_t n_items;
    int32_t n_tiles;      // total tiles
    int64_t n_slots;      // total record slots
    int64_t n_pixels;     // total pixels
};

// Item owning record slot `slot` / global tile `tile` (tables are ordered by
// g_off and tile_off).  Uniform when the argument is.
__device__ __forceinline__ int item_of_slot(const Item* items, int n_items, int64_t slot) {
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].g_off <= slot) lo = mid; else hi = mid - 1;
    }
    return lo;
}
__device__ __forceinline__ int item_of_tile(const Item* items, int n_items, int tile) {
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].tile_off <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------- launchers
// (each returns hipSuccess or the launch error)

// With `totals`, also zeroes the frame counts (before launch_preprocess adds to them).
hipError_t write_items(Item* table, const Item* host_items, int n_items, hipStream_t s,
                       uint64_t* totals = nullptr);
// A second stream the colour kernel can run on while the caller's stream goes
// on with the stages that do not read the colour: `fork` is recorded on the
// caller's stream after the geometry kernel and waited for by `stream`;
// `join` is recorded on `stream` after the colour kernel, and the caller's
// stream must wait for it before anything reads frame.rgb.
struct SideStream {
    hipStream_t stream;
    hipEvent_t fork, join;
};
// sh_rows16: every item's SH rows start 16-byte aligned (base aligned and a
// row of a multiple of 4 floats), so the colour kernel can load rows whole.
// side: run the colour kernel there (null: on s).  host_single (a frame of one
// item, d.n_items == 1): the item, which the geometry kernel takes as an
// argument and writes to `table` (== items) while zeroing the frame counts,
// in place of write_items.
hipError_t launch_preprocess(const Item* items, const BatchDims& d, int mode, const ss_frame& f,
                             bool sh_rows16, hipStream_t s, const SideStream* side = nullptr,
                             const Item* host_single = nullptr, Item* table = nullptr);
// With `totals` (device frame counts) non-null, n_visible, n, n_entries and
// n_pairs below are bounds and the stages read their counts from `totals`.
hipError_t launch_depth_order(int64_t n, int64_t n_visible, const ss_frame& f, hipStream_t s,
                              const uint64_t* totals = nullptr);
hipError_t launch_scan(int64_t n, const ss_frame& f, hipStream_t s,
                       const uint64_t* totals = nullptr);
int64_t scan_tmp_words(int64_t n);
int64_t emit_tmp_words(int64_t n);
hipError_t launch_emit(const Item* items, const BatchDims& d, int mode, const ss_frame& f,
                       int64_t n_entries, uint32_t* keys, uint32_t* values, uint64_t n_pairs,
                       hipStream_t s, const uint64_t* totals = nullptr);
int64_t sort_tmp_words(uint64_t capacity);
int sort_passes(int bits);
hipError_t launch_sort(const ss_pairs& p, int buf, uint64_t n_pairs, int bits, int* out_buf,
                       hipStream_t s, const uint64_t* totals = nullptr);
// launch_sort with the sort scratch in the library's static device array (the
// caller's p.sort_tmp is not used): hipErrorInvalidValue if the pass needs more
// than static_sort_tmp_words(), or the runtime's error looking it up.
hipError_t launch_sort_static(const ss_pairs& p, int buf, uint64_t n_pairs, int bits,
                              int* out_buf, hipStream_t s);
int64_t static_sort_tmp_words();
hipError_t launch_ranges(const uint32_t* keys, uint64_t n_pairs, int n_tiles, uint32_t* ranges,
                         hipStream_t s, const uint64_t* totals = nullptr);
// launch_blend = launch_tile_order (the tiles' work order, from the ranges)
// followed by launch_blend_tiles.
// counts_out: host memory the device can write (or null), receives the frame
// counts f.totals[0..1] when the tile order runs.
hipError_t launch_tile_order(const Item* items, const BatchDims& d, const ss_frame& f,
                             hipStream_t s, uint64_t* counts_out = nullptr);
// persistent: a resident grid pulling tiles from per-XCD work queues instead of
// one workgroup per tile (the same results).
hipError_t launch_blend_tiles(const Item* items, const BatchDims& d, const ss_frame& f,
                              const uint32_t* values, float* out_rgb_single, hipStream_t s,
                              bool persistent = false);
hipError_t launch_blend(const Item* items, const BatchDims& d, const ss_frame& f,
                        const uint32_t* values, float* out_rgb_single, hipStream_t s,
                        bool persistent = false);
int64_t prune_tmp_words(int64_t n);
// Kept indices (ascending) of the n_keep highest scores, ties to the lower index.
hipError_t launch_prune_select(const float* score, int64_t n, int64_t n_keep, uint32_t* keep_idx,
                               uint32_t* tmp, hipStream_t s);
// dst[j, :] = src[idx[j], :] for rows of w floats, j < m.
hipError_t launch_gather(const float* src, const uint32_t* idx, int64_t m, int w, float* dst,
                         hipStream_t s);
hipError_t launch_backward(const ss_camera& cam, const ss_gaussians& g, const ss_frame& f,
                           const uint32_t* values, const float* dl_drgb, const ss_grads& out,
                           void* const* ev, hipStream_t s);

}  // namespace ss

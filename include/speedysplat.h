/*
 * speedysplat.h - C ABI of the MI355X (gfx950) Speedy-Splat rasterizer.
 *
 * The library renders a set of 3D Gaussians G_i = {mu_i, s_i, r_i, h_i,
 * sigma_i} for a camera pose (Speedy-Splat, arXiv 2412.00578, Sec. 3.1) with the
 * tile-based pipeline of Sec. 3.2.1-3.2.3 and one of three tile assignments:
 *   SS_TILE_3SIGMA    the square of radius ceil(3 sqrt(lambda_max)) (Eq. radius)
 *   SS_TILE_SNUGBOX   the opacity-aware tight bounding box (Sec. 4.1.1)
 *   SS_TILE_ACCUTILE  the exact tiles touched by the ellipse (Sec. 4.1.2, Alg. 1)
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every array argument is DEVICE memory owned by the caller, C-contiguous,
 *   at least 16-byte aligned (torch allocations are).  The library never
 *   allocates or frees device memory and keeps no state between calls other
 *   than its loaded kernels and the static scratch array of ss_sort_noalloc.
 * - `stream` is a hipStream_t (NULL = the null stream).  Every call only
 *   enqueues work on it and returns; outputs are valid once the stream has
 *   been synchronised.  The exceptions, which synchronise `stream` to read the
 *   frame counts, are named "SYNC" below.
 * - Status: SS_OK (0) or a positive SS_ERR_* code.  Arguments are checked on
 *   the host before anything is enqueued; on an error nothing is enqueued and
 *   ss_last_error() holds a message (thread-local).  A launch failure reported
 *   by the HIP runtime returns SS_ERR_HIP.
 * - Data-dependent degeneracies are not errors: a Gaussian that is not finite,
 *   lies at or before the near plane, has a non-positive-definite screen
 *   covariance, or (SnugBox/AccuTile) an opacity <= 1/255 is culled: its record
 *   is all zeros and its tile count 0.
 *
 * Geometry conventions
 * --------------------
 * Camera: x_cam = R x_world + t, +z forward, +x right, +y down; pinhole
 * u = fx x/z + cx, v = fy y/z + cy.  Pixel (px, py) is sampled at its centre
 * (px + 0.5, py + 0.5); tile (tx, ty) covers [16 tx, 16 tx + 16) x
 * [16 ty, 16 ty + 16); tiles_x = ceil(W/16), tiles_y = ceil(H/16),
 * tile id = ty * tiles_x + tx.
 *
 * Per-Gaussian record (written by the preprocess stage, read by the rest):
 *   geom  [n,4] f32 = (u, v, depth, t)      t = 2 ln(255 sigma)  (Sec. 4.1)
 *   conic [n,4] f32 = (a, b, c, sigma)      Sigma_2D^{-1} = [[a, b], [b, c]]
 *   rgb   [n,4] f32 = (r, g, b, 0)          view-dependent SH colour
 * geom and conic are interleaved in one [n,8] buffer: Gaussian i's geom is
 * floats 8i .. 8i+3 of frame->geom and its conic floats 8i+4 .. 8i+7, with
 * frame->conic == frame->geom + 4 (a record gather then touches 32
 * contiguous bytes).
 * The geometry is evaluated in FP64 from the FP32 inputs and rounded once into
 * the record; every tile decision is then made in FP64 on the stored record, so
 * the tile counts of the preprocess stage equal the pairs the emit stage writes.
 *
 * Pair order (Sec. 3.2.2).  The paper sorts (key, value) pairs with key =
 * (uint64 tile_id << 32) | bits(depth as f32) and value = Gaussian index; the
 * sorted order is by tile, then depth, then index.  This library reaches the
 * same order in two stable sorts: ss_depth_order sorts the Gaussians by
 * bits(depth) (ties by index), ss_emit writes the pairs in that order with
 * key = tile id (uint32), and ss_sort sorts them stably on the tile id.
 */
#ifndef SPEEDYSPLAT_H
#define SPEEDYSPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SS_ABI_VERSION 5

enum ss_status {
    SS_OK = 0,
    SS_ERR_INVALID_ARG = 1, /* null pointer, bad size, degree or mode */
    SS_ERR_WORKSPACE = 2,   /* pair workspace smaller than the pair count */
    SS_ERR_OVERFLOW = 3,    /* more than 2^32 - 1 pairs, or too many tiles */
    SS_ERR_HIP = 4          /* the HIP runtime reported an error */
};

enum ss_tile_mode { SS_TILE_3SIGMA = 0, SS_TILE_SNUGBOX = 1, SS_TILE_ACCUTILE = 2 };

/* Constants the kernels use, exported so tests can compare them with their
 * own independently typed copies. */
typedef struct ss_constants {
    int32_t abi_version;
    int32_t tile;          /* 16 (Sec. 3.2: 16 x 16 pixel tiles) */
    float alpha_min;       /* 1/255: inclusion cutoff (Sec. 3.2.3) */
    float alpha_max;       /* 0.99: upper clamp of alpha */
    float t_min;           /* 1e-4: transmittance stop */
    float dilation;        /* 0.3 added to the diagonal of Sigma_2D */
    float fov_clamp;       /* 1.3: x/z, y/z clamp in the EWA Jacobian, in half-FOV units */
    float disc_floor;      /* 0.1: floor of the eigenvalue discriminant (3-sigma) */
} ss_constants;

typedef struct ss_camera {
    int32_t width, height;  /* pixels, 1 .. 16384 */
    float fx, fy, cx, cy;   /* pinhole intrinsics, pixels */
    float R[9];             /* world -> camera rotation, row-major */
    float t[3];             /* world -> camera translation */
    float near_z;           /* cull depth (z <= near_z is culled) */
    float bg[3];            /* background colour added with the final T */
} ss_camera;

typedef struct ss_gaussians {
    int64_t n;              /* number of Gaussians, 0 .. 2^31 - 1 */
    int32_t sh_degree;      /* 0 .. 3 */
    int32_t sh_stride;      /* coefficients stored per Gaussian, >= (deg+1)^2 */
    const float *means;     /* [n,3] world positions mu_i */
    const float *scales;    /* [n,3] linear scales s_i (the activation is the caller's) */
    const float *quats;     /* [n,4] rotations r_i as (w, x, y, z), any non-zero norm */
    const float *opacity;   /* [n]   sigma_i in (0, 1] */
    const float *sh;        /* [n, sh_stride, 3] SH coefficients h_i */
} ss_gaussians;

/* Per-frame buffers, sized by ss_frame_sizes(). */
typedef struct ss_frame {
    float *geom;            /* [n,8] (geom, conic) records, 16-byte aligned (32 keeps
                               each record within one 64-byte line) */
    float *conic;           /* geom + 4 (rejected otherwise) */
    float *rgb;             /* [n,4] */
    uint32_t *counts;       /* [n]   tiles per Gaussian */
    uint32_t *depth_keys;   /* [2n]  depth-order sort keys: the preprocess stage writes
                               [0, n) (bits(depth), or 0xffffffff for a Gaussian with no
                               tiles); [n, 2n) is scratch of ss_depth_order */
    uint32_t *order;        /* [2n]  after ss_depth_order, [0, n_visible) holds the
                               Gaussians with tiles sorted by (depth key, index);
                               [n, 2n) is scratch */
    uint32_t *order_counts; /* [n]   after ss_depth_order: the tile count of order[j]
                               (tile_sets[order[j]] word 3), j < n_visible */
    uint32_t *order_tmp;    /* [order_tmp_words] scratch of ss_depth_order */
    uint32_t *tile_sets;    /* [n,4] per Gaussian, written by the preprocess stage: when
                               its tile rectangle fits 8 x 8 tiles, the 64-bit mask
                               (words 0-1, bit r * 8 + c = tile (x0 + c, y0 + r)) and
                               x0 | y0 << 16 (word 2); mask 0 otherwise; word 3 is the
                               tile count */
    uint32_t *offsets;      /* [n]   inclusive prefix sum of counts in depth order */
    uint64_t *scan_tmp;     /* [scan_tmp_words]; word 0 receives the pair count P */
    uint64_t *totals;       /* [2] the frame counts (ss_frame_counts: P, Gaussians with
                               tiles), zeroed and accumulated by the preprocess stage */
    uint32_t *ranges;       /* [n_tiles, 2] 8-byte aligned: per-tile [start, end) into the
                               sorted pairs */
    float *t_final;         /* [H, W] final transmittance per pixel */
    uint32_t *n_last;       /* [H, W] 1 + position (within its tile) of the last
                               Gaussian blended into the pixel, 0 if none */
    uint32_t *n_eval;       /* optional [H, W] (NULL: not written): Gaussians of the
                               tile's list the pixel evaluated before it stopped */
    uint32_t *n_contrib;    /* optional [H, W], written only with n_eval: Gaussians
                               blended into the pixel */
    uint32_t *emit_tmp;     /* [emit_tmp_words] 16-byte aligned: scratch of the preprocess
                               stage (partial frame counts), the depth order (which
                               leaves the tile sets in depth order at its start for the
                               emit stage) and the emit stage (queue of Gaussians with
                               many tiles); contents are not an output */
    void *table;            /* [table_bytes] 16-byte aligned: the frame's item table
                               (camera, scene pointers, offsets), written by
                               ss_preprocess / ss_forward_begin / ss_batch_begin and
                               read by the later stages of the same frame, then the
                               blend's tile work order (written by the blend stage) */
} ss_frame;

typedef struct ss_frame_info {
    int32_t tiles_x, tiles_y, n_tiles;
    int32_t sort_bits;      /* significant tile-key bits: ceil(log2(n_tiles)) */
    int64_t scan_tmp_words; /* uint64 words for ss_frame.scan_tmp */
    int64_t order_tmp_words; /* uint32 words for ss_frame.order_tmp */
    int64_t emit_tmp_words; /* uint32 words for ss_frame.emit_tmp */
    int64_t table_bytes;    /* bytes for ss_frame.table */
} ss_frame_info;

/* The frame counts the preprocess stage accumulates and the begin calls read
 * back: the pair count P (the sum of the tile counts) and the number of
 * Gaussians with at least one tile. */
typedef struct ss_frame_counts {
    uint64_t n_pairs;
    uint64_t n_visible;
} ss_frame_counts;

/* One render request of a batch: a camera, a resident scene, an output image. */
typedef struct ss_batch_item {
    ss_camera cam;
    ss_gaussians g;         /* device pointers of a scene (shared between items freely) */
    float *out_rgb;         /* [3, H, W] f32 device image this item's blend writes */
} ss_batch_item;

/* Buffer sizes of a batch (ss_batch_sizes).  The frame of a batch holds all
 * items: per-Gaussian buffers have n_slots entries (each item's records start
 * at a multiple of 256), per-pixel buffers n_pixels (items' pixels packed in
 * order), ranges n_tiles rows (items' tiles packed in order). */
typedef struct ss_batch_info {
    int64_t n_slots;
    int64_t n_pixels;
    int32_t n_tiles;
    int32_t sort_bits;      /* ceil(log2(n_tiles)) */
    int64_t scan_tmp_words;
    int64_t order_tmp_words;
    int64_t emit_tmp_words;
    int64_t table_bytes;
} ss_batch_info;

/* Pair workspace: two ping-pong key/value buffers plus sort scratch. */
typedef struct ss_pairs {
    uint64_t capacity;      /* pairs each buffer holds */
    uint32_t *keys[2];      /* [capacity] each: tile ids */
    uint32_t *values[2];    /* [capacity] each */
    uint32_t *sort_tmp;     /* [sort_tmp_words] */
} ss_pairs;

/* Gradients written by ss_render_backward (device memory, caller-owned). */
typedef struct ss_grads {
    float *means;           /* [n,3]  dL/dmu (overwritten) */
    float *scales;          /* [n,3]  dL/ds for the linear scales (overwritten) */
    float *quats;           /* [n,4]  dL/dr for the quaternions as given (overwritten) */
    float *opacity;         /* [n]    dL/dsigma (overwritten) */
    float *sh;              /* [n, sh_stride, 3] dL/dh (overwritten; unused degrees 0) */
    float *g2d;             /* [n,12] screen-space gradients, also scratch: per Gaussian
                               (du, dv, 0, 0, da, db, dc, dsigma, dr, dg, db, 0) */
    float *score;           /* optional [n] (NULL: skipped): sum over pixels and channels
                               of (dC/dg_i)^2, g_i the 2D Gaussian's value at the pixel */
} ss_grads;

/* Optional stage timing for the composite calls: caller-created hipEvent_t
 * handles (NULL entries are skipped) recorded on the stream at
 *   [0] before preprocess  [1] after preprocess  [2] before the depth order
 *   (after the frame counts were read back)  [3] after the depth order
 *   [4] after the scan  [5] after emit  [6] after the sort  [7] after the ranges
 *   and the tiles' work order  [8] after the blend, so [7]..[8] brackets the
 *   blend kernel alone. */
typedef struct ss_stage_events {
    void *ev[9];
} ss_stage_events;

/* Fills *out.  Returns SS_ERR_INVALID_ARG for a null pointer. */
int ss_get_constants(ss_constants *out);

/* Static message for a status code (never NULL). */
const char *ss_status_string(int status);

/* Message of the last failing call on this thread ("" if none). */
const char *ss_last_error(void);

/* Buffer sizes for a frame of n Gaussians at width x height. */
int ss_frame_sizes(int64_t n, int32_t width, int32_t height, ss_frame_info *out);

/* uint32 words of ss_pairs.sort_tmp for `capacity` pairs. */
int ss_sort_tmp_words(uint64_t capacity, int64_t *out_words);

/*
 * Stage 1, preprocess (Sec. 3.2.1 and Sec. 4.1): for every Gaussian, the record
 * (projection, Sigma_3D = R S S^T R^T, EWA Sigma_2D + 0.3 I, conic, t, SH
 * colour) and its tile count under `mode`.  Writes frame->geom, conic, rgb,
 * counts, tile_sets and depth_keys[0, n), and the frame counts (P and the
 * number of Gaussians with tiles) to frame->totals.
 */
int ss_preprocess(const ss_camera *cam, const ss_gaussians *g, int32_t mode,
                  const ss_frame *frame, void *stream);

/*
 * Stage 2a, depth order (the depth half of the Sec. 3.2.2 sort key): stable LSD
 * radix sort of the Gaussians with tiles on frame->depth_keys (the n keys the
 * preprocess stage wrote, of which n_visible differ from 0xffffffff);
 * frame->order[0, n_visible) receives their indices by (bits(depth), index),
 * frame->order_counts[j] the tile count of order[j] and emit_tmp (as [n, 4])
 * the tile set of order[j], both read from tile_sets[order[j]].  The first
 * pass drops the Gaussians without tiles, so later passes sort n_visible keys.
 * Uses depth_keys[0, 2n), order[n, 2n) and order_tmp as scratch.
 */
int ss_depth_order(int64_t n, int64_t n_visible, const ss_frame *frame, void *stream);

/*
 * Stage 2b, inclusive prefix sum of the tile counts in depth order (Sec. 3.2.2,
 * "InclusiveSum"): frame->offsets[j] = sum_{k <= j} order_counts[k] for
 * j < n_visible; the total P goes to frame->scan_tmp[0] (uint64).
 */
int ss_scan(int64_t n_visible, const ss_frame *frame, void *stream);

/*
 * Stage 3, key emission (Sec. 3.2.2, "duplicateWithKeys"; Alg. 1 "Process"):
 * for each depth-order entry j < n_visible, Gaussian i = order[j] writes its
 * tiles (in an unspecified order) at [offsets[j] - counts[i], offsets[j]) of
 * pairs->keys[buf] (tile id) / values[buf] (i), reading its tile set from the
 * depth-ordered copy ss_depth_order left in emit_tmp.  n is the number of
 * Gaussians; n_pairs must be the P the scan produced and <= pairs->capacity.
 */
int ss_emit(const ss_camera *cam, int64_t n, int64_t n_visible, int32_t mode,
            const ss_frame *frame, const ss_pairs *pairs, int32_t buf, uint64_t n_pairs,
            void *stream);

/*
 * Stage 4, LSD radix sort of the pairs in buffer `buf` on the low
 * ss_frame_info.sort_bits bits of the tile key (Sec. 3.2.2, "RadixSort"); stable,
 * so a tile's pairs keep their depth order.  *out_buf receives the buffer
 * holding the result.
 */
int ss_sort(const ss_camera *cam, const ss_pairs *pairs, int32_t buf, uint64_t n_pairs,
            int32_t *out_buf, void *stream);

/*
 * ss_sort for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * sort, arguments, result and errors, but the sort's scratch (one pass's
 * per-workgroup digit counts and digit totals) lives in a static device array
 * of the library, 1 MiB + 1 KiB on each GPU it runs on, held until the
 * process ends; pairs->sort_tmp is not read and may be NULL.  The keys and
 * values buffers are still the caller's.  The scratch needed does not grow
 * with the pair count (at most 2^32 - 2 pairs, as for ss_sort); a larger need
 * would return SS_ERR_WORKSPACE.  The first call on a device looks up the
 * array's address for that device (the current device, which must be the
 * stream's).  Calls that overlap on one GPU share the array and race:
 * serialise them (one stream, or events).  Allocates nothing.
 */
int ss_sort_noalloc(const ss_camera *cam, const ss_pairs *pairs, int32_t buf, uint64_t n_pairs,
                    int32_t *out_buf, void *stream);

/*
 * Stage 5, per-tile ranges of the sorted keys (Sec. 3.2.2, "identifyTileRanges"):
 * frame->ranges[tile] = [first, last + 1) of the tile's run; an empty tile gets
 * start = end = the position where its run would begin.
 */
int ss_ranges(const ss_camera *cam, const ss_frame *frame, const ss_pairs *pairs, int32_t buf,
              uint64_t n_pairs, void *stream);

/*
 * Stage 6, blend (Sec. 3.2.3, Eqs. render_alpha, 2d_gaussian_scalar,
 * contribution): front to back over each tile's sorted Gaussians, a Gaussian
 * is included at a pixel when q <= t (alpha >= 1/255), alpha = min(0.99,
 * sigma exp(-q/2)); the walk stops before a Gaussian that would take the
 * transmittance below 1e-4.  out_rgb is planar [3, H, W] f32; also writes
 * frame->t_final and frame->n_last.  Tiles are processed longest list first
 * (the order is written into frame->table after the item table); the result
 * does not depend on the order.
 */
int ss_blend(const ss_camera *cam, const ss_frame *frame, const ss_pairs *pairs, int32_t buf,
             float *out_rgb, void *stream);

/*
 * SYNC.  Stage 1, then reads the frame counts back to the host (*counts_out).
 * Returns SS_ERR_OVERFLOW if P >= 2^32.  `events` may be NULL.
 */
int ss_forward_begin(const ss_camera *cam, const ss_gaussians *g, int32_t mode,
                     const ss_frame *frame, ss_frame_counts *counts_out,
                     const ss_stage_events *events, void *stream);

/*
 * Stage 1 like ss_forward_begin, without waiting: the frame counts are copied
 * into the HOST struct *counts_host by a copy enqueued on `stream` after the
 * preprocess stage, and the call returns at once.  *counts_host is valid once
 * the stream has passed that copy (synchronise an event recorded after this
 * call).  Pinned host memory (hipHostMalloc) keeps the copy asynchronous.  The
 * caller then grows the pair workspace if needed and calls ss_forward_finish;
 * meanwhile it may enqueue other frames' work, e.g. the next frame's stage 1
 * into a second ss_frame, so that the GPU never waits for the host.
 */
int ss_forward_begin_async(const ss_camera *cam, const ss_gaussians *g, int32_t mode,
                           const ss_frame *frame, ss_frame_counts *counts_host,
                           const ss_stage_events *events, void *stream);

/*
 * Stages 2a-6 for the frame counts returned by ss_forward_begin (or
 * ss_forward_begin_async).  Returns SS_ERR_WORKSPACE if pairs->capacity <
 * counts->n_pairs.  *out_buf (may be NULL) receives the pair buffer holding the
 * sorted pairs.  `events` may be NULL.
 */
int ss_forward_finish(const ss_camera *cam, int64_t n, int32_t mode, const ss_frame *frame,
                      const ss_pairs *pairs, const ss_frame_counts *counts, float *out_rgb,
                      int32_t *out_buf, const ss_stage_events *events, void *stream);

/*
 * Stages 3-6 (emit, sort, ranges, blend) of ss_forward_finish, for a frame
 * whose stage 2a and 2 the caller has already run (ss_depth_order with the
 * frame's n and counts->n_visible, then ss_scan), possibly on another stream
 * ordered before this one: a pipeline can then run frame k + 1's depth order
 * beside frame k's blend.  Same arguments, results and errors as
 * ss_forward_finish; events [2]..[4] are recorded together at the start.
 */
int ss_forward_back(const ss_camera *cam, int64_t n, int32_t mode, const ss_frame *frame,
                    const ss_pairs *pairs, const ss_frame_counts *counts, float *out_rgb,
                    int32_t *out_buf, const ss_stage_events *events, void *stream);

/*
 * SYNC.  The whole forward render (stages 1-6).  *counts_out (may be NULL)
 * receives the frame counts.  If pairs->capacity < P, returns SS_ERR_WORKSPACE
 * after stage 1 without touching the pair buffers; the caller grows them to P
 * and calls again.  `events` may be NULL.
 *
 * ss_render, ss_render_nosync and ss_render_band run the colour kernel on a
 * second stream of the library's (one per device, created on first use, held
 * until the process ends) while `stream` runs the depth order, scan, emit,
 * sort and ranges; `stream` waits for it before the blend, and also when the
 * call fails after it started.  Work queued on `stream` after the call is
 * therefore ordered after every kernel of the frame, as with a single stream.
 * Calls from several host threads on one device are serialised inside the
 * library while they queue their work.  Stage event [1] follows the geometry
 * kernel: the colour kernel's time falls within stages 2a-5.
 */
int ss_render(const ss_camera *cam, const ss_gaussians *g, int32_t mode, const ss_frame *frame,
              const ss_pairs *pairs, float *out_rgb, ss_frame_counts *counts_out,
              int32_t *out_buf, const ss_stage_events *events, void *stream);

/*
 * The whole forward render (stages 1-6) with no host synchronisation: the
 * stages after the preprocess are launched over upper bounds (the record
 * slots, pairs->capacity) and read the frame counts the preprocess stage
 * leaves in frame->totals on the device, so the host can queue frame after
 * frame and the GPU never waits for a read-back.  If the frame has more pairs
 * than pairs->capacity, no pair is written and the image is the background
 * alone: the caller finds out from the frame counts, which land in
 * *counts_host (host memory; may be NULL) by the time the stream has run the
 * frame, and renders the frame again with a larger workspace.  Page-locked
 * host memory (hipHostMalloc, or registered with the runtime) is written by a
 * kernel of the frame; other host memory by a copy enqueued after the
 * preprocess stage.  Otherwise the results equal ss_render's bit for bit.
 * pairs->capacity must be at least 1; *out_buf receives the pair buffer
 * holding the sorted pairs.  Events as for ss_render (event [2] directly
 * follows [1]: there is no read-back).
 */
int ss_render_nosync(const ss_camera *cam, const ss_gaussians *g, int32_t mode,
                     const ss_frame *frame, const ss_pairs *pairs, float *out_rgb,
                     ss_frame_counts *counts_host, int32_t *out_buf,
                     const ss_stage_events *events, void *stream);

/*
 * SYNC.  The forward render of one band of tile rows [tile_row0, tile_row0 +
 * tile_rows) of the camera's image: the piece of a frame one GPU renders
 * when a frame is split across GPUs by screen-space bands (the tile pipeline
 * of Sec. 3.2 restricted to a viewport).  Every Gaussian is preprocessed for
 * the whole camera, exactly as by ss_render; only tiles in the band's rows
 * are counted, emitted, sorted, given ranges and blended, and the band's
 * tile ids, per-pixel buffers and image are relative to its first row:
 * tile id = (ty - tile_row0) * tiles_x + tx, pixel row py - 16 tile_row0.
 * The band's pairs, ranges and pixels equal the whole frame's restricted to
 * the band, bit for bit.  `frame` is sized by ss_frame_sizes(n, width,
 * band_height), band_height = min(height, 16 (tile_row0 + tile_rows)) -
 * 16 tile_row0, and out_rgb is [3, band_height, width].  Errors as for
 * ss_render (SS_ERR_WORKSPACE with *counts_out set when the pair workspace is
 * too small), and SS_ERR_INVALID_ARG for a band outside the image.  The
 * adjoint (ss_render_backward) takes whole frames only.
 */
int ss_render_band(const ss_camera *cam, const ss_gaussians *g, int32_t mode, int32_t tile_row0,
                   int32_t tile_rows, const ss_frame *frame, const ss_pairs *pairs,
                   float *out_rgb, ss_frame_counts *counts_out, int32_t *out_buf,
                   const ss_stage_events *events, void *stream);

/* Sizes for a batch of n_items (1 .. 4096) items. */
int ss_batch_sizes(const ss_batch_item *items, int32_t n_items, ss_batch_info *out);

/*
 * SYNC.  Batched stage 1 for n_items render requests (different scenes and
 * resolutions) in one launch: the item table is written to frame->table,
 * records go to the items' slots, and the frame counts of the whole batch
 * are read back.  Pair keys carry a batch-global tile id (the
 * item's first tile + its tile), so one depth order and one tile sort order
 * every item's tiles, and an item's pairs, sorted and blended, are those it
 * would have alone.
 */
int ss_batch_begin(const ss_batch_item *items, int32_t n_items, int32_t mode,
                   const ss_frame *frame, ss_frame_counts *counts_out,
                   const ss_stage_events *events, void *stream);

/*
 * Batched stages 2a-6 for the counts returned by ss_batch_begin (same items,
 * mode and frame); each item's image goes to its out_rgb.  Returns
 * SS_ERR_WORKSPACE if pairs->capacity < counts->n_pairs.
 */
int ss_batch_finish(const ss_batch_item *items, int32_t n_items, int32_t mode,
                    const ss_frame *frame, const ss_pairs *pairs,
                    const ss_frame_counts *counts, int32_t *out_buf,
                    const ss_stage_events *events, void *stream);

/*
 * Adjoint of the forward render (the gradient flow of Sec. 4.2: per-pixel
 * gradients aggregated to the 2D parameters, then per Gaussian to the 3D
 * ones).  Inputs: the same camera and Gaussians as the forward call, its
 * frame (records, ranges, t_final, n_last) and pair workspace (`buf` holds
 * the sorted pairs), and dl_drgb [3, H, W], the loss gradient of the image.
 * The blend is walked back to front per tile, recomputing alpha and the
 * transmittance from the stored final T.  out->g2d and out->score are
 * zeroed and accumulated with FP32 atomics (their summation order varies
 * between runs); the parameter gradients are then written per Gaussian.
 * Culled Gaussians get zero gradients.  `events` (may be NULL) are recorded
 * at [0] the start, [1] after zeroing g2d and score, [2] after the blend
 * adjoint (stage 7), [3] after the preprocess adjoint (stage 8).
 */
int ss_render_backward(const ss_camera *cam, const ss_gaussians *g, const ss_frame *frame,
                       const ss_pairs *pairs, int32_t buf, const float *dl_drgb,
                       const ss_grads *out, const ss_stage_events *events, void *stream);

/*
 * Pruning (Sec. 4.2.2 Soft Pruning: a fraction of the Gaussians removed at
 * scheduled points of training; Sec. 4.2.3 Hard Pruning: a constant fraction
 * removed at fixed intervals), ranked by the efficient pruning score of
 * Sec. 4.2.1 (ss_grads.score, summed over the views the caller chooses).
 *
 * ss_prune_count: *n_keep_out = n - floor(prune_ratio * n), the product taken
 * in double precision; prune_ratio in [0, 1].
 * ss_prune_tmp_words: uint32 words of scratch for ss_prune_select.
 * ss_prune_select: keep_idx[0, n_keep) receives, in ascending order, the
 * indices of the n_keep highest scores; a score that is NaN or <= 0 ranks as
 * 0, and among equal scores at the threshold the lower indices are kept.
 * score [n] f32, keep_idx [n_keep] u32 and tmp are device memory; n_keep is
 * known on the host when the call returns (no synchronisation).
 * ss_gather_gaussians: compacts the Gaussians to the kept ones: every
 * parameter row j of `out` (n = n_keep, the input's SH degree and stride,
 * caller-owned device arrays) receives row keep_idx[j] of `in`.
 */
int ss_prune_count(int64_t n, double prune_ratio, int64_t *n_keep_out);
int ss_prune_tmp_words(int64_t n, int64_t *out_words);
int ss_prune_select(const float *score, int64_t n, double prune_ratio, uint32_t *keep_idx,
                    uint32_t *tmp, int64_t *n_keep_out, void *stream);
int ss_gather_gaussians(const ss_gaussians *in, const uint32_t *keep_idx, int64_t n_keep,
                        const ss_gaussians *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SPEEDYSPLAT_H */

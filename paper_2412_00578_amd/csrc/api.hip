// C ABI of the library (declared in include/speedysplat.h): argument checks on
// the host, then asynchronous launches on the caller's stream.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "ss_internal.h"

namespace {

thread_local char g_err[512] = "";

int fail(int status, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return status;
}

int hip_status(hipError_t e, const char* where) {
    if (e == hipSuccess) return SS_OK;
    return fail(SS_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

int tiles_of(const ss_camera* cam, int* tx, int* ty) {
    *tx = (cam->width + ss::kTile - 1) / ss::kTile;
    *ty = (cam->height + ss::kTile - 1) / ss::kTile;
    return *tx * *ty;
}

int sort_bits_for(int n_tiles) {
    int b = 0;
    while ((1ll << b) < (long long)n_tiles) ++b;
    return 32 + b;
}

int check_camera(const ss_camera* cam) {
    if (!cam) return fail(SS_ERR_INVALID_ARG, "camera is NULL");
    if (cam->width < 1 || cam->height < 1 || cam->width > 16384 || cam->height > 16384)
        return fail(SS_ERR_INVALID_ARG, "image size %dx%d outside 1..16384", cam->width,
                    cam->height);
    if (!(cam->fx > 0.0f) || !(cam->fy > 0.0f))
        return fail(SS_ERR_INVALID_ARG, "focal lengths must be positive");
    return SS_OK;
}

int check_gaussians(const ss_gaussians* g) {
    if (!g) return fail(SS_ERR_INVALID_ARG, "gaussians is NULL");
    if (g->n < 0 || g->n > 0x7fffffffll)
        return fail(SS_ERR_INVALID_ARG, "n = %lld outside 0..2^31-1", (long long)g->n);
    if (g->sh_degree < 0 || g->sh_degree > 3)
        return fail(SS_ERR_INVALID_ARG, "sh_degree %d outside 0..3", g->sh_degree);
    if (g->sh_stride < (g->sh_degree + 1) * (g->sh_degree + 1))
        return fail(SS_ERR_INVALID_ARG, "sh_stride %d < (deg+1)^2", g->sh_stride);
    if (g->n > 0 && (!g->means || !g->scales || !g->quats || !g->opacity || !g->sh))
        return fail(SS_ERR_INVALID_ARG, "a Gaussian parameter pointer is NULL");
    if (g->n > 0 && (!aligned16(g->quats) || !aligned16(g->sh)))
        return fail(SS_ERR_INVALID_ARG, "quats and sh must be 16-byte aligned");
    return SS_OK;
}

int check_mode(int32_t mode) {
    if (mode < SS_TILE_3SIGMA || mode > SS_TILE_ACCUTILE)
        return fail(SS_ERR_INVALID_ARG, "tile mode %d is not 0, 1 or 2", mode);
    return SS_OK;
}

int check_frame_records(const ss_frame* f, int64_t n) {
    if (!f) return fail(SS_ERR_INVALID_ARG, "frame is NULL");
    if (n > 0 && (!f->geom || !f->conic || !f->rgb || !f->counts || !f->offsets || !f->emit_tmp))
        return fail(SS_ERR_INVALID_ARG, "a per-Gaussian frame buffer is NULL");
    if (!aligned16(f->geom) || !aligned16(f->conic) || !aligned16(f->rgb))
        return fail(SS_ERR_INVALID_ARG, "frame records must be 16-byte aligned");
    if (!f->scan_tmp) return fail(SS_ERR_INVALID_ARG, "frame scan_tmp is NULL");
    return SS_OK;
}

int check_frame_pixels(const ss_frame* f) {
    if (!f->ranges || !f->t_final || !f->n_last)
        return fail(SS_ERR_INVALID_ARG, "a per-tile or per-pixel frame buffer is NULL");
    return SS_OK;
}

int check_pairs(const ss_pairs* p, int32_t buf, uint64_t n_pairs) {
    if (!p) return fail(SS_ERR_INVALID_ARG, "pairs is NULL");
    if (buf != 0 && buf != 1) return fail(SS_ERR_INVALID_ARG, "pair buffer %d is not 0 or 1", buf);
    if (n_pairs > p->capacity)
        return fail(SS_ERR_WORKSPACE, "%llu pairs exceed the workspace capacity %llu",
                    (unsigned long long)n_pairs, (unsigned long long)p->capacity);
    if (n_pairs >= 0xffffffffull)
        return fail(SS_ERR_OVERFLOW, "%llu pairs do not fit 32-bit offsets",
                    (unsigned long long)n_pairs);
    if (p->capacity > 0 && (!p->keys[0] || !p->keys[1] || !p->values[0] || !p->values[1] ||
                            !p->sort_tmp))
        return fail(SS_ERR_INVALID_ARG, "a pair workspace pointer is NULL");
    return SS_OK;
}

void record(const ss_stage_events* ev, int k, hipStream_t s) {
    if (ev && ev->ev[k]) (void)hipEventRecord((hipEvent_t)ev->ev[k], s);
}

#define SS_TRY(x)                      \
    do {                               \
        int _st = (x);                 \
        if (_st != SS_OK) return _st;  \
    } while (0)

}  // namespace

extern "C" {

int ss_get_constants(ss_constants* out) {
    if (!out) return fail(SS_ERR_INVALID_ARG, "out is NULL");
    out->abi_version = SS_ABI_VERSION;
    out->tile = ss::kTile;
    out->alpha_min = ss::kAlphaMin;
    out->alpha_max = ss::kAlphaMax;
    out->t_min = ss::kTMin;
    out->dilation = (float)ss::kDilation;
    out->fov_clamp = (float)ss::kFovClamp;
    out->disc_floor = (float)ss::kDiscFloor;
    return SS_OK;
}

const char* ss_status_string(int status) {
    switch (status) {
        case SS_OK: return "ok";
        case SS_ERR_INVALID_ARG: return "invalid argument";
        case SS_ERR_WORKSPACE: return "pair workspace too small";
        case SS_ERR_OVERFLOW: return "pair count overflow";
        case SS_ERR_HIP: return "HIP runtime error";
        default: return "unknown status";
    }
}

const char* ss_last_error(void) { return g_err; }

int ss_frame_sizes(int64_t n, int32_t width, int32_t height, ss_frame_info* out) {
    if (!out) return fail(SS_ERR_INVALID_ARG, "out is NULL");
    if (n < 0 || width < 1 || height < 1 || width > 16384 || height > 16384)
        return fail(SS_ERR_INVALID_ARG, "bad frame size");
    out->tiles_x = (width + ss::kTile - 1) / ss::kTile;
    out->tiles_y = (height + ss::kTile - 1) / ss::kTile;
    out->n_tiles = out->tiles_x * out->tiles_y;
    out->sort_bits = sort_bits_for(out->n_tiles);
    out->scan_tmp_words = ss::scan_tmp_words(n);
    return SS_OK;
}

int ss_sort_tmp_words(uint64_t capacity, int64_t* out_words) {
    if (!out_words) return fail(SS_ERR_INVALID_ARG, "out is NULL");
    *out_words = ss::sort_tmp_words(capacity);
    return SS_OK;
}

int ss_preprocess(const ss_camera* cam, const ss_gaussians* g, int32_t mode, const ss_frame* f,
                  void* stream) {
    SS_TRY(check_camera(cam));
    SS_TRY(check_gaussians(g));
    SS_TRY(check_mode(mode));
    SS_TRY(check_frame_records(f, g->n));
    return hip_status(ss::launch_preprocess(*cam, *g, mode, *f, (hipStream_t)stream),
                      "preprocess");
}

int ss_scan(int64_t n, const ss_frame* f, void* stream) {
    if (n < 0) return fail(SS_ERR_INVALID_ARG, "n < 0");
    SS_TRY(check_frame_records(f, n));
    return hip_status(ss::launch_scan(n, *f, (hipStream_t)stream), "scan");
}

int ss_emit(const ss_camera* cam, int64_t n, int32_t mode, const ss_frame* f, const ss_pairs* p,
            int32_t buf, uint64_t n_pairs, void* stream) {
    SS_TRY(check_camera(cam));
    SS_TRY(check_mode(mode));
    if (n < 0) return fail(SS_ERR_INVALID_ARG, "n < 0");
    SS_TRY(check_frame_records(f, n));
    SS_TRY(check_pairs(p, buf, n_pairs));
    int tx, ty;
    tiles_of(cam, &tx, &ty);
    return hip_status(ss::launch_emit(tx, ty, n, mode, *f, p->keys[buf], p->values[buf], n_pairs,
                                      (hipStream_t)stream),
                      "emit");
}

int ss_sort(const ss_camera* cam, const ss_pairs* p, int32_t buf, uint64_t n_pairs,
            int32_t* out_buf, void* stream) {
    SS_TRY(check_camera(cam));
    SS_TRY(check_pairs(p, buf, n_pairs));
    if (!out_buf) return fail(SS_ERR_INVALID_ARG, "out_buf is NULL");
    int tx, ty;
    const int bits = sort_bits_for(tiles_of(cam, &tx, &ty));
    int ob = buf;
    int st = hip_status(ss::launch_sort(*p, buf, n_pairs, bits, &ob, (hipStream_t)stream), "sort");
    *out_buf = ob;
    return st;
}

int ss_ranges(const ss_camera* cam, const ss_frame* f, const ss_pairs* p, int32_t buf,
              uint64_t n_pairs, void* stream) {
    SS_TRY(check_camera(cam));
    if (!f) return fail(SS_ERR_INVALID_ARG, "frame is NULL");
    SS_TRY(check_frame_pixels(f));
    SS_TRY(check_pairs(p, buf, n_pairs));
    int tx, ty;
    const int n_tiles = tiles_of(cam, &tx, &ty);
    return hip_status(ss::launch_ranges(p->keys[buf], n_pairs, n_tiles, f->ranges,
                                        (hipStream_t)stream),
                      "ranges");
}

int ss_blend(const ss_camera* cam, const ss_frame* f, const ss_pairs* p, int32_t buf,
             float* out_rgb, void* stream) {
    SS_TRY(check_camera(cam));
    if (!f) return fail(SS_ERR_INVALID_ARG, "frame is NULL");
    SS_TRY(check_frame_pixels(f));
    if (!p || (buf != 0 && buf != 1)) return fail(SS_ERR_INVALID_ARG, "bad pair workspace");
    if (!out_rgb) return fail(SS_ERR_INVALID_ARG, "out_rgb is NULL");
    if (!aligned16(f->geom) || !aligned16(f->conic) || !aligned16(f->rgb))
        return fail(SS_ERR_INVALID_ARG, "frame records must be 16-byte aligned");
    return hip_status(ss::launch_blend(*cam, *f, p->values[buf], out_rgb, (hipStream_t)stream),
                      "blend");
}

int ss_forward_begin(const ss_camera* cam, const ss_gaussians* g, int32_t mode, const ss_frame* f,
                     uint64_t* n_pairs_out, const ss_stage_events* ev, void* stream) {
    if (!n_pairs_out) return fail(SS_ERR_INVALID_ARG, "n_pairs_out is NULL");
    hipStream_t s = (hipStream_t)stream;
    record(ev, 0, s);
    SS_TRY(ss_preprocess(cam, g, mode, f, stream));
    record(ev, 1, s);
    SS_TRY(ss_scan(g->n, f, stream));
    record(ev, 2, s);
    uint64_t p = 0;
    SS_TRY(hip_status(hipMemcpyAsync(&p, f->scan_tmp, sizeof(p), hipMemcpyDeviceToHost, s),
                      "read pair count"));
    SS_TRY(hip_status(hipStreamSynchronize(s), "synchronise"));
    *n_pairs_out = p;
    if (p >= 0xffffffffull)
        return fail(SS_ERR_OVERFLOW, "%llu pairs do not fit 32-bit offsets", (unsigned long long)p);
    return SS_OK;
}

int ss_forward_finish(const ss_camera* cam, int64_t n, int32_t mode, const ss_frame* f,
                      const ss_pairs* p, uint64_t n_pairs, float* out_rgb, int32_t* out_buf,
                      const ss_stage_events* ev, void* stream) {
    SS_TRY(check_camera(cam));
    SS_TRY(check_mode(mode));
    SS_TRY(check_frame_records(f, n));
    SS_TRY(check_frame_pixels(f));
    SS_TRY(check_pairs(p, 0, n_pairs));
    if (!out_rgb) return fail(SS_ERR_INVALID_ARG, "out_rgb is NULL");
    int tx, ty;
    const int n_tiles = tiles_of(cam, &tx, &ty);
    const int bits = sort_bits_for(n_tiles);
    hipStream_t s = (hipStream_t)stream;
    // Emit into the buffer that makes the sorted result land in buffer 0.
    const int passes = n_pairs > 1 ? ss::sort_passes(bits) : 0;
    const int first = passes & 1;
    record(ev, 3, s);
    SS_TRY(hip_status(
        ss::launch_emit(tx, ty, n, mode, *f, p->keys[first], p->values[first], n_pairs, s), "emit"));
    record(ev, 4, s);
    int cur = first;
    SS_TRY(hip_status(ss::launch_sort(*p, first, n_pairs, bits, &cur, s), "sort"));
    record(ev, 5, s);
    SS_TRY(hip_status(ss::launch_ranges(p->keys[cur], n_pairs, n_tiles, f->ranges, s), "ranges"));
    record(ev, 6, s);
    SS_TRY(hip_status(ss::launch_blend(*cam, *f, p->values[cur], out_rgb, s), "blend"));
    record(ev, 7, s);
    if (out_buf) *out_buf = cur;
    return SS_OK;
}

int ss_render(const ss_camera* cam, const ss_gaussians* g, int32_t mode, const ss_frame* f,
              const ss_pairs* p, float* out_rgb, uint64_t* n_pairs_out, int32_t* out_buf,
              const ss_stage_events* ev, void* stream) {
    if (!p) return fail(SS_ERR_INVALID_ARG, "pairs is NULL");
    uint64_t n_pairs = 0;
    SS_TRY(ss_forward_begin(cam, g, mode, f, &n_pairs, ev, stream));
    if (n_pairs_out) *n_pairs_out = n_pairs;
    if (n_pairs > p->capacity)
        return fail(SS_ERR_WORKSPACE, "%llu pairs exceed the workspace capacity %llu",
                    (unsigned long long)n_pairs, (unsigned long long)p->capacity);
    return ss_forward_finish(cam, g->n, mode, f, p, n_pairs, out_rgb, out_buf, ev, stream);
}

int ss_render_backward(const ss_camera* cam, const ss_gaussians* g, const ss_frame* f,
                       const ss_pairs* p, int32_t buf, const float* dl_drgb, const ss_grads* out,
                       void* stream) {
    SS_TRY(check_camera(cam));
    SS_TRY(check_gaussians(g));
    SS_TRY(check_frame_records(f, g->n));
    SS_TRY(check_frame_pixels(f));
    if (!p || (buf != 0 && buf != 1)) return fail(SS_ERR_INVALID_ARG, "bad pair workspace");
    if (!dl_drgb) return fail(SS_ERR_INVALID_ARG, "dl_drgb is NULL");
    if (!out) return fail(SS_ERR_INVALID_ARG, "grads is NULL");
    if (g->n > 0 && (!out->means || !out->scales || !out->quats || !out->opacity || !out->sh ||
                     !out->g2d))
        return fail(SS_ERR_INVALID_ARG, "a gradient buffer is NULL");
    return hip_status(
        ss::launch_backward(*cam, *g, *f, p->values[buf], dl_drgb, *out, (hipStream_t)stream),
        "backward");
}

}  // extern "C"

// C ABI of the library (declared in include/speedysplat.h): argument checks on
// the host, then asynchronous launches on the caller's stream.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

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

// The colour kernel's second stream and its two events, one set per device,
// created on first use (default priority, not synchronising with the null
// stream) and held until the process ends.  A single-call render holds its
// device's lock from the fork to the enqueued join, so calls from several
// host threads do not interleave the events.
struct DeviceSide {
    std::mutex mu;
    ss::SideStream side{nullptr, nullptr, nullptr};
    bool ready = false;
};
constexpr int kMaxSideDevices = 64;
DeviceSide g_side[kMaxSideDevices];

int side_for_device(DeviceSide** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e, "get device");
    if (dev < 0 || dev >= kMaxSideDevices) return fail(SS_ERR_HIP, "device %d out of range", dev);
    DeviceSide& d = g_side[dev];
    std::lock_guard<std::mutex> lock(d.mu);
    if (!d.ready) {
        e = hipStreamCreateWithFlags(&d.side.stream, hipStreamNonBlocking);
        // both ends of each dependency run on this device: no system-scope
        // fence (a writeback of the L2s) when the events are recorded
        const unsigned flags = hipEventDisableTiming | hipEventDisableSystemFence;
        if (e == hipSuccess) e = hipEventCreateWithFlags(&d.side.fork, flags);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&d.side.join, flags);
        if (e != hipSuccess) return hip_status(e, "colour stream");
        d.ready = true;
    }
    *out = &d;
    return SS_OK;
}

int tiles_of(const ss_camera* cam, int* tx, int* ty) {
    *tx = (cam->width + ss::kTile - 1) / ss::kTile;
    *ty = (cam->height + ss::kTile - 1) / ss::kTile;
    return *tx * *ty;
}

// Bits of the tile sort: ceil(log2(n_tiles)) (the depth half of the paper's
// key is ordered by the depth-order stage).
int sort_bits_for(int n_tiles) {
    int b = 0;
    while ((1ll << b) < (long long)n_tiles) ++b;
    return b;
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
    if (n > 0 && (!f->geom || !f->conic || !f->rgb || !f->counts || !f->offsets || !f->emit_tmp ||
                  !f->depth_keys || !f->order || !f->order_counts || !f->order_tmp ||
                  !f->tile_sets))
        return fail(SS_ERR_INVALID_ARG, "a per-Gaussian frame buffer is NULL");
    if (!f->totals) return fail(SS_ERR_INVALID_ARG, "frame totals is NULL");
    if (n > 0 && f->conic != f->geom + 4)
        return fail(SS_ERR_INVALID_ARG, "frame conic must be frame geom + 4 (interleaved records)");
    if (!aligned16(f->geom) || !aligned16(f->conic) || !aligned16(f->rgb) ||
        !aligned16(f->tile_sets) || !aligned16(f->emit_tmp))
        return fail(SS_ERR_INVALID_ARG, "frame records and emit_tmp must be 16-byte aligned");
    if (!f->scan_tmp) return fail(SS_ERR_INVALID_ARG, "frame scan_tmp is NULL");
    return SS_OK;
}

int check_frame_pixels(const ss_frame* f) {
    if (!f->ranges || !f->t_final || !f->n_last)
        return fail(SS_ERR_INVALID_ARG, "a per-tile or per-pixel frame buffer is NULL");
    if (((uintptr_t)f->ranges & 7u) != 0)
        return fail(SS_ERR_INVALID_ARG, "frame ranges must be 8-byte aligned");
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

constexpr int kMaxItems = 4096;
#ifndef SS_PERSISTENT_FRAMES
#define SS_PERSISTENT_FRAMES 0
#endif
constexpr bool kPersistentFrames = SS_PERSISTENT_FRAMES != 0;

int64_t pad_slots(int64_t n) { return (n + ss::kSlotAlign - 1) / ss::kSlotAlign * ss::kSlotAlign; }

// Host copy of a batch's item table and its totals.
struct Layout {
    std::vector<ss::Item> items;
    ss::BatchDims d{};
};

// Every item's SH rows start 16-byte aligned.
bool sh_rows16(const Layout& L) {
    for (const ss::Item& it : L.items)
        if (((uintptr_t)it.sh & 15u) != 0 || ((3 * it.sh_stride) & 3) != 0) return false;
    return true;
}

ss::Item make_item(const ss_camera& cam, const ss_gaussians& g, float* out) {
    ss::Item it{};
    it.cam = cam;
    it.means = g.means; it.scales = g.scales; it.quats = g.quats;
    it.opacity = g.opacity; it.sh = g.sh; it.out_rgb = out;
    it.n = g.n;
    it.sh_degree = g.sh_degree; it.sh_stride = g.sh_stride;
    it.tx_n = (cam.width + ss::kTile - 1) / ss::kTile;
    it.ty_n = (cam.height + ss::kTile - 1) / ss::kTile;
    it.by0 = 0;
    it.by1 = it.ty_n;
    return it;
}

// Places the items one after another: record slots padded to 256, tiles and
// pixels packed.
int lay_out(const ss_batch_item* items, int n_items, Layout& L) {
    if (!items || n_items < 1 || n_items > kMaxItems)
        return fail(SS_ERR_INVALID_ARG, "a batch holds 1..%d items", kMaxItems);
    L.items.resize((size_t)n_items);
    int64_t slots = 0, pixels = 0, tiles = 0;
    for (int k = 0; k < n_items; ++k) {
        SS_TRY(check_camera(&items[k].cam));
        SS_TRY(check_gaussians(&items[k].g));
        ss::Item it = make_item(items[k].cam, items[k].g, items[k].out_rgb);
        it.g_off = slots;
        it.tile_off = (int32_t)tiles;
        it.pix_off = pixels;
        slots += pad_slots(it.n);
        tiles += (int64_t)it.tx_n * it.ty_n;
        pixels += (int64_t)it.cam.width * it.cam.height;
        L.items[(size_t)k] = it;
    }
    if (tiles >= (1ll << 31) || slots >= (1ll << 32) - 1)
        return fail(SS_ERR_OVERFLOW, "batch too large (%lld tiles, %lld slots)",
                    (long long)tiles, (long long)slots);
    L.d.n_items = n_items;
    L.d.n_tiles = (int32_t)tiles;
    L.d.n_slots = slots;
    L.d.n_pixels = pixels;
    return SS_OK;
}

Layout single_layout(const ss_camera& cam, const ss_gaussians& g) {
    Layout L;
    L.items.push_back(make_item(cam, g, nullptr));
    L.d.n_items = 1;
    L.d.n_tiles = L.items[0].tx_n * L.items[0].ty_n;
    L.d.n_slots = g.n;
    L.d.n_pixels = (int64_t)cam.width * cam.height;
    return L;
}

// A single frame restricted to the tile rows [row0, row0 + rows): every
// Gaussian is preprocessed, but only the band's tiles get pairs, and the
// per-tile and per-pixel buffers and the image cover the band's rows.
Layout band_layout(const ss_camera& cam, const ss_gaussians& g, int row0, int rows) {
    Layout L = single_layout(cam, g);
    ss::Item& it = L.items[0];
    it.by0 = row0;
    it.by1 = row0 + rows;
    const int y_end = cam.height < it.by1 * ss::kTile ? cam.height : it.by1 * ss::kTile;
    L.d.n_tiles = it.tx_n * rows;
    L.d.n_pixels = (int64_t)cam.width * (y_end - row0 * ss::kTile);
    return L;
}

// Dims of a single frame when only the camera and n are at hand.
ss::BatchDims single_dims(const ss_camera& cam, int64_t n) {
    ss::BatchDims d{};
    int tx, ty;
    d.n_items = 1;
    d.n_tiles = tiles_of(&cam, &tx, &ty);
    d.n_slots = n;
    d.n_pixels = (int64_t)cam.width * cam.height;
    return d;
}

int check_table(const ss_frame* f) {
    if (!f || !f->table) return fail(SS_ERR_INVALID_ARG, "frame table is NULL");
    if (((uintptr_t)f->table & 15u) != 0)
        return fail(SS_ERR_INVALID_ARG, "frame table must be 16-byte aligned");
    return SS_OK;
}

// Stage 1 and the read-back of the frame counts (P, visible Gaussians).
// sync: wait and store them in *out; otherwise enqueue their copy into the
// host struct *out and return.
int begin_impl(const Layout& L, int32_t mode, const ss_frame* f, ss_frame_counts* out,
               const ss_stage_events* ev, bool sync, hipStream_t s,
               const ss::SideStream* side = nullptr) {
    SS_TRY(check_mode(mode));
    SS_TRY(check_frame_records(f, L.d.n_slots));
    SS_TRY(check_table(f));
    if (!out && sync) return fail(SS_ERR_INVALID_ARG, "frame counts pointer is NULL");
    ss::Item* table = reinterpret_cast<ss::Item*>(f->table);
    record(ev, 0, s);
    // a single item travels with the geometry kernel
    const bool single = L.d.n_items == 1;
    if (!single)
        SS_TRY(hip_status(ss::write_items(table, L.items.data(), L.d.n_items, s, f->totals),
                          "item table"));
    SS_TRY(hip_status(ss::launch_preprocess(table, L.d, mode, *f, sh_rows16(L), s, side,
                                            single ? L.items.data() : nullptr, table),
                      "preprocess"));
    record(ev, 1, s);
    static_assert(sizeof(ss_frame_counts) == 2 * sizeof(uint64_t), "counts layout");
    if (!sync)
        return out ? hip_status(hipMemcpyAsync(out, f->totals, sizeof(ss_frame_counts),
                                               hipMemcpyDeviceToHost, s),
                                "copy frame counts")
                   : SS_OK;
    ss_frame_counts c{};
    SS_TRY(hip_status(hipMemcpyAsync(&c, f->totals, sizeof(c), hipMemcpyDeviceToHost, s),
                      "read frame counts"));
    SS_TRY(hip_status(hipStreamSynchronize(s), "synchronise"));
    *out = c;
    if (c.n_pairs >= 0xffffffffull)
        return fail(SS_ERR_OVERFLOW, "%llu pairs do not fit 32-bit offsets",
                    (unsigned long long)c.n_pairs);
    return SS_OK;
}

// Stages 2a-6 for the counts begin_impl returned; with order false, stages
// 3-6 only (the caller ran the depth order and the scan).  With c == NULL the
// stages read the frame counts on the device (frame->totals), launched over
// the record slots and the pair workspace's capacity (no host read-back).
// counts_dev: host memory the device can write (or null), receives the frame
// counts from the tile-order kernel.
int finish_impl(const ss::BatchDims& d, int32_t mode, const ss_frame* f, const ss_pairs* p,
                const ss_frame_counts* c, float* out_single, int32_t* out_buf,
                const ss_stage_events* ev, hipStream_t s, bool order = true,
                uint64_t* counts_dev = nullptr, const ss::SideStream* side = nullptr) {
    SS_TRY(check_mode(mode));
    SS_TRY(check_frame_records(f, d.n_slots));
    SS_TRY(check_frame_pixels(f));
    SS_TRY(check_table(f));
    const uint64_t* totals = nullptr;
    uint64_t n_pairs;
    int64_t n_vis;
    if (c) {
        if (c->n_visible > (uint64_t)d.n_slots)
            return fail(SS_ERR_INVALID_ARG, "n_visible %llu exceeds the %lld record slots",
                        (unsigned long long)c->n_visible, (long long)d.n_slots);
        n_pairs = c->n_pairs;
        n_vis = (int64_t)c->n_visible;
        SS_TRY(check_pairs(p, 0, n_pairs));
    } else {
        if (!p) return fail(SS_ERR_INVALID_ARG, "pairs is NULL");
        if (p->capacity < 1)
            return fail(SS_ERR_WORKSPACE, "the pair workspace has no capacity");
        n_pairs = p->capacity;             // bounds; the counts are read on the device
        n_vis = d.n_slots;
        SS_TRY(check_pairs(p, 0, n_pairs));
        totals = f->totals;
    }
    const ss::Item* table = reinterpret_cast<const ss::Item*>(f->table);
    const int bits = sort_bits_for(d.n_tiles);
    // Emit into the buffer that makes the sorted result land in buffer 0.
    const int passes = (n_pairs > 1 || totals) ? ss::sort_passes(bits) : 0;
    const int first = passes & 1;
    record(ev, 2, s);
    if (order)
        SS_TRY(hip_status(ss::launch_depth_order(d.n_slots, n_vis, *f, s, totals), "depth order"));
    record(ev, 3, s);
    if (order) SS_TRY(hip_status(ss::launch_scan(n_vis, *f, s, totals), "scan"));
    record(ev, 4, s);
    SS_TRY(hip_status(ss::launch_emit(table, d, mode, *f, n_vis, p->keys[first],
                                      p->values[first], n_pairs, s, totals),
                      "emit"));
    record(ev, 5, s);
    int cur = first;
    SS_TRY(hip_status(ss::launch_sort(*p, first, n_pairs, bits, &cur, s, totals), "sort"));
    record(ev, 6, s);
    SS_TRY(hip_status(ss::launch_ranges(p->keys[cur], n_pairs, d.n_tiles, f->ranges, s, totals),
                      "ranges"));
    SS_TRY(hip_status(ss::launch_tile_order(table, d, *f, s, counts_dev), "tile order"));
    // the colour (run on the side stream) is read from here on; the blend
    // stage's event follows the wait, so the stage times the blend alone
    if (side) SS_TRY(hip_status(hipStreamWaitEvent(s, side->join, 0), "join colour stream"));
    record(ev, 7, s);
    // a batch's tiles (every item, every resolution) are served by one resident
    // grid pulling from per-XCD work queues
    const bool persistent = d.n_items > 1 || kPersistentFrames;
    SS_TRY(hip_status(ss::launch_blend_tiles(table, d, *f, p->values[cur], out_single, s,
                                             persistent),
                      "blend"));
    record(ev, 8, s);
    if (out_buf) *out_buf = cur;
    return SS_OK;
}

// A whole frame in one call, with the colour kernel on the device's side
// stream while the caller's stream runs the depth order, scan, emit, sort and
// ranges; body(side) runs begin_impl and finish_impl, which waits for the
// colour before the blend.  If a step fails after the fork, the caller's
// stream still waits for the colour, so nothing queued later on it can race
// the colour kernel's writes.
template <class Body>
int with_colour_stream(hipStream_t s, Body body) {
    DeviceSide* ds = nullptr;
    SS_TRY(side_for_device(&ds));
    std::lock_guard<std::mutex> lock(ds->mu);
    const int st = body(static_cast<const ss::SideStream*>(&ds->side));
    if (st != SS_OK) (void)hipStreamWaitEvent(s, ds->side.join, 0);
    return st;
}

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
    out->order_tmp_words = ss::sort_tmp_words((uint64_t)n);
    out->emit_tmp_words = ss::emit_tmp_words(n);
    out->table_bytes = ss::table_bytes(1, out->n_tiles);
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
    SS_TRY(check_table(f));
    const Layout L = single_layout(*cam, *g);
    hipStream_t s = (hipStream_t)stream;
    ss::Item* table = reinterpret_cast<ss::Item*>(f->table);
    return hip_status(ss::launch_preprocess(table, L.d, mode, *f, sh_rows16(L), s, nullptr,
                                            L.items.data(), table),
                      "preprocess");
}

int ss_depth_order(int64_t n, int64_t n_visible, const ss_frame* f, void* stream) {
    if (n < 0 || n_visible < 0 || n_visible > n)
        return fail(SS_ERR_INVALID_ARG, "need 0 <= n_visible <= n");
    SS_TRY(check_frame_records(f, n));
    return hip_status(ss::launch_depth_order(n, n_visible, *f, (hipStream_t)stream),
                      "depth order");
}

int ss_scan(int64_t n_visible, const ss_frame* f, void* stream) {
    if (n_visible < 0) return fail(SS_ERR_INVALID_ARG, "n_visible < 0");
    SS_TRY(check_frame_records(f, n_visible));
    return hip_status(ss::launch_scan(n_visible, *f, (hipStream_t)stream), "scan");
}

int ss_emit(const ss_camera* cam, int64_t n, int64_t n_visible, int32_t mode, const ss_frame* f,
            const ss_pairs* p, int32_t buf, uint64_t n_pairs, void* stream) {
    SS_TRY(check_camera(cam));
    SS_TRY(check_mode(mode));
    if (n < 0 || n_visible < 0 || n_visible > n)
        return fail(SS_ERR_INVALID_ARG, "need 0 <= n_visible <= n");
    SS_TRY(check_frame_records(f, n));
    SS_TRY(check_table(f));
    SS_TRY(check_pairs(p, buf, n_pairs));
    return hip_status(ss::launch_emit(reinterpret_cast<const ss::Item*>(f->table),
                                      single_dims(*cam, n), mode, *f, n_visible, p->keys[buf],
                                      p->values[buf], n_pairs, (hipStream_t)stream),
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

int ss_sort_noalloc(const ss_camera* cam, const ss_pairs* p, int32_t buf, uint64_t n_pairs,
                    int32_t* out_buf, void* stream) {
    SS_TRY(check_camera(cam));
    if (!p) return fail(SS_ERR_INVALID_ARG, "pairs is NULL");
    ss_pairs q = *p;
    q.sort_tmp = reinterpret_cast<uint32_t*>(q.keys[0]);   // unused; satisfies the NULL check
    SS_TRY(check_pairs(&q, buf, n_pairs));
    if (!out_buf) return fail(SS_ERR_INVALID_ARG, "out_buf is NULL");
    if (ss::sort_tmp_words(n_pairs) > ss::static_sort_tmp_words())
        return fail(SS_ERR_WORKSPACE,
                    "sorting %llu pairs needs %lld scratch words; the static scratch holds %lld",
                    (unsigned long long)n_pairs, (long long)ss::sort_tmp_words(n_pairs),
                    (long long)ss::static_sort_tmp_words());
    int tx, ty;
    const int bits = sort_bits_for(tiles_of(cam, &tx, &ty));
    int ob = buf;
    int st = hip_status(ss::launch_sort_static(q, buf, n_pairs, bits, &ob, (hipStream_t)stream),
                        "sort (static scratch)");
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
    SS_TRY(check_table(f));
    if (!p || (buf != 0 && buf != 1)) return fail(SS_ERR_INVALID_ARG, "bad pair workspace");
    if (!out_rgb) return fail(SS_ERR_INVALID_ARG, "out_rgb is NULL");
    if (!aligned16(f->geom) || !aligned16(f->conic) || !aligned16(f->rgb))
        return fail(SS_ERR_INVALID_ARG, "frame records must be 16-byte aligned");
    return hip_status(ss::launch_blend(reinterpret_cast<const ss::Item*>(f->table),
                                       single_dims(*cam, 0), *f, p->values[buf], out_rgb,
                                       (hipStream_t)stream),
                      "blend");
}

int ss_forward_begin(const ss_camera* cam, const ss_gaussians* g, int32_t mode, const ss_frame* f,
                     ss_frame_counts* counts_out, const ss_stage_events* ev, void* stream) {
    SS_TRY(check_camera(cam));
    SS_TRY(check_gaussians(g));
    return begin_impl(single_layout(*cam, *g), mode, f, counts_out, ev, true,
                      (hipStream_t)stream);
}

int ss_forward_begin_async(const ss_camera* cam, const ss_gaussians* g, int32_t mode,
                           const ss_frame* f, ss_frame_counts* counts_host,
                           const ss_stage_events* ev, void* stream) {
    SS_TRY(check_camera(cam));
    SS_TRY(check_gaussians(g));
    return begin_impl(single_layout(*cam, *g), mode, f, counts_host, ev, false,
                      (hipStream_t)stream);
}

int ss_forward_finish(const ss_camera* cam, int64_t n, int32_t mode, const ss_frame* f,
                      const ss_pairs* p, const ss_frame_counts* counts, float* out_rgb,
                      int32_t* out_buf, const ss_stage_events* ev, void* stream) {
    SS_TRY(check_camera(cam));
    if (n < 0) return fail(SS_ERR_INVALID_ARG, "n < 0");
    if (!out_rgb) return fail(SS_ERR_INVALID_ARG, "out_rgb is NULL");
    return finish_impl(single_dims(*cam, n), mode, f, p, counts, out_rgb, out_buf, ev,
                       (hipStream_t)stream);
}

int ss_forward_back(const ss_camera* cam, int64_t n, int32_t mode, const ss_frame* f,
                    const ss_pairs* p, const ss_frame_counts* counts, float* out_rgb,
                    int32_t* out_buf, const ss_stage_events* ev, void* stream) {
    SS_TRY(check_camera(cam));
    if (n < 0) return fail(SS_ERR_INVALID_ARG, "n < 0");
    if (!out_rgb) return fail(SS_ERR_INVALID_ARG, "out_rgb is NULL");
    return finish_impl(single_dims(*cam, n), mode, f, p, counts, out_rgb, out_buf, ev,
                       (hipStream_t)stream, false);
}

int ss_render(const ss_camera* cam, const ss_gaussians* g, int32_t mode, const ss_frame* f,
              const ss_pairs* p, float* out_rgb, ss_frame_counts* counts_out, int32_t* out_buf,
              const ss_stage_events* ev, void* stream) {
    if (!p) return fail(SS_ERR_INVALID_ARG, "pairs is NULL");
    SS_TRY(check_camera(cam));
    SS_TRY(check_gaussians(g));
    if (!out_rgb) return fail(SS_ERR_INVALID_ARG, "out_rgb is NULL");
    const Layout L = single_layout(*cam, *g);
    const hipStream_t s = (hipStream_t)stream;
    return with_colour_stream(s, [&](const ss::SideStream* side) {
        ss_frame_counts c{};
        SS_TRY(begin_impl(L, mode, f, &c, ev, true, s, side));
        if (counts_out) *counts_out = c;
        if (c.n_pairs > p->capacity)
            return fail(SS_ERR_WORKSPACE, "%llu pairs exceed the workspace capacity %llu",
                        (unsigned long long)c.n_pairs, (unsigned long long)p->capacity);
        return finish_impl(L.d, mode, f, p, &c, out_rgb, out_buf, ev, s, true, nullptr, side);
    });
}

int ss_render_nosync(const ss_camera* cam, const ss_gaussians* g, int32_t mode,
                     const ss_frame* f, const ss_pairs* p, float* out_rgb,
                     ss_frame_counts* counts_host, int32_t* out_buf, const ss_stage_events* ev,
                     void* stream) {
    SS_TRY(check_camera(cam));
    SS_TRY(check_gaussians(g));
    if (!out_rgb) return fail(SS_ERR_INVALID_ARG, "out_rgb is NULL");
    const Layout L = single_layout(*cam, *g);
    const hipStream_t s = (hipStream_t)stream;
    // Page-locked host memory is written by the tile-order kernel (no copy on
    // the stream); other host memory by a copy after the preprocess stage.
    uint64_t* counts_dev = nullptr;
    if (counts_host && L.d.n_tiles > 0) {     // the tile-order kernel runs
        hipPointerAttribute_t attr{};
        if (hipPointerGetAttributes(&attr, counts_host) == hipSuccess &&
            attr.type == hipMemoryTypeHost && attr.devicePointer && attr.hostPointer)
            // the device address of counts_host itself (the attributes may
            // describe the start of its allocation)
            counts_dev = reinterpret_cast<uint64_t*>(
                static_cast<char*>(attr.devicePointer) +
                (reinterpret_cast<char*>(counts_host) - static_cast<char*>(attr.hostPointer)));
        else
            (void)hipGetLastError();     // not registered with the runtime
    }
    return with_colour_stream(s, [&](const ss::SideStream* side) {
        SS_TRY(begin_impl(L, mode, f, counts_dev ? nullptr : counts_host, ev, false, s, side));
        return finish_impl(L.d, mode, f, p, nullptr, out_rgb, out_buf, ev, s, true, counts_dev,
                           side);
    });
}

int ss_render_band(const ss_camera* cam, const ss_gaussians* g, int32_t mode, int32_t tile_row0,
                   int32_t tile_rows, const ss_frame* f, const ss_pairs* p, float* out_rgb,
                   ss_frame_counts* counts_out, int32_t* out_buf, const ss_stage_events* ev,
                   void* stream) {
    SS_TRY(check_camera(cam));
    SS_TRY(check_gaussians(g));
    if (!p) return fail(SS_ERR_INVALID_ARG, "pairs is NULL");
    if (!out_rgb) return fail(SS_ERR_INVALID_ARG, "out_rgb is NULL");
    int tx, ty;
    tiles_of(cam, &tx, &ty);
    if (tile_row0 < 0 || tile_row0 >= ty || tile_rows < 1 || tile_rows > ty - tile_row0)
        return fail(SS_ERR_INVALID_ARG, "band rows [%d, %d) outside the %d tile rows",
                    tile_row0, tile_row0 + tile_rows, ty);
    const Layout L = band_layout(*cam, *g, tile_row0, tile_rows);
    const hipStream_t s = (hipStream_t)stream;
    return with_colour_stream(s, [&](const ss::SideStream* side) {
        ss_frame_counts c{};
        SS_TRY(begin_impl(L, mode, f, &c, ev, true, s, side));
        if (counts_out) *counts_out = c;
        if (c.n_pairs > p->capacity)
            return fail(SS_ERR_WORKSPACE, "%llu pairs exceed the workspace capacity %llu",
                        (unsigned long long)c.n_pairs, (unsigned long long)p->capacity);
        return finish_impl(L.d, mode, f, p, &c, out_rgb, out_buf, ev, s, true, nullptr, side);
    });
}

int ss_batch_sizes(const ss_batch_item* items, int32_t n_items, ss_batch_info* out) {
    if (!out) return fail(SS_ERR_INVALID_ARG, "out is NULL");
    Layout L;
    SS_TRY(lay_out(items, n_items, L));
    out->n_slots = L.d.n_slots;
    out->n_pixels = L.d.n_pixels;
    out->n_tiles = L.d.n_tiles;
    out->sort_bits = sort_bits_for(L.d.n_tiles);
    out->scan_tmp_words = ss::scan_tmp_words(L.d.n_slots);
    out->order_tmp_words = ss::sort_tmp_words((uint64_t)L.d.n_slots);
    out->emit_tmp_words = ss::emit_tmp_words(L.d.n_slots);
    out->table_bytes = ss::table_bytes(n_items, L.d.n_tiles);
    return SS_OK;
}

int ss_batch_begin(const ss_batch_item* items, int32_t n_items, int32_t mode, const ss_frame* f,
                   ss_frame_counts* counts_out, const ss_stage_events* ev, void* stream) {
    Layout L;
    SS_TRY(lay_out(items, n_items, L));
    for (int k = 0; k < n_items; ++k)
        if (!items[k].out_rgb) return fail(SS_ERR_INVALID_ARG, "item %d has no out_rgb", k);
    return begin_impl(L, mode, f, counts_out, ev, true, (hipStream_t)stream);
}

int ss_batch_finish(const ss_batch_item* items, int32_t n_items, int32_t mode, const ss_frame* f,
                    const ss_pairs* p, const ss_frame_counts* counts, int32_t* out_buf,
                    const ss_stage_events* ev, void* stream) {
    Layout L;
    SS_TRY(lay_out(items, n_items, L));
    return finish_impl(L.d, mode, f, p, counts, nullptr, out_buf, ev, (hipStream_t)stream);
}

int ss_prune_tmp_words(int64_t n, int64_t* out_words) {
    if (!out_words) return fail(SS_ERR_INVALID_ARG, "out is NULL");
    if (n < 0 || n > 0x7fffffffll) return fail(SS_ERR_INVALID_ARG, "n outside 0..2^31-1");
    *out_words = ss::prune_tmp_words(n);
    return SS_OK;
}

int ss_prune_count(int64_t n, double prune_ratio, int64_t* n_keep_out) {
    if (!n_keep_out) return fail(SS_ERR_INVALID_ARG, "n_keep_out is NULL");
    if (n < 0 || n > 0x7fffffffll) return fail(SS_ERR_INVALID_ARG, "n outside 0..2^31-1");
    if (!(prune_ratio >= 0.0 && prune_ratio <= 1.0))
        return fail(SS_ERR_INVALID_ARG, "prune ratio %g outside [0, 1]", prune_ratio);
    const double pruned = floor(prune_ratio * (double)n);
    *n_keep_out = n - (int64_t)pruned;
    return SS_OK;
}

int ss_prune_select(const float* score, int64_t n, double prune_ratio, uint32_t* keep_idx,
                    uint32_t* tmp, int64_t* n_keep_out, void* stream) {
    int64_t n_keep = 0;
    SS_TRY(ss_prune_count(n, prune_ratio, &n_keep));
    if (n > 0 && (!score || !tmp || (n_keep > 0 && !keep_idx)))
        return fail(SS_ERR_INVALID_ARG, "a pruning buffer is NULL");
    *n_keep_out = n_keep;
    return hip_status(ss::launch_prune_select(score, n, n_keep, keep_idx, tmp, (hipStream_t)stream),
                      "prune select");
}

int ss_gather_gaussians(const ss_gaussians* in, const uint32_t* keep_idx, int64_t n_keep,
                        const ss_gaussians* out, void* stream) {
    SS_TRY(check_gaussians(in));
    if (!out) return fail(SS_ERR_INVALID_ARG, "out is NULL");
    if (n_keep < 0 || n_keep > in->n)
        return fail(SS_ERR_INVALID_ARG, "n_keep %lld outside 0..%lld", (long long)n_keep,
                    (long long)in->n);
    if (out->n != n_keep || out->sh_degree != in->sh_degree || out->sh_stride != in->sh_stride)
        return fail(SS_ERR_INVALID_ARG, "out must have n = n_keep and the input's SH layout");
    if (n_keep == 0) return SS_OK;
    if (!keep_idx || !out->means || !out->scales || !out->quats || !out->opacity || !out->sh)
        return fail(SS_ERR_INVALID_ARG, "a gather buffer is NULL");
    const hipStream_t s = (hipStream_t)stream;
    SS_TRY(hip_status(ss::launch_gather(in->means, keep_idx, n_keep, 3, (float*)out->means, s),
                      "gather means"));
    SS_TRY(hip_status(ss::launch_gather(in->scales, keep_idx, n_keep, 3, (float*)out->scales, s),
                      "gather scales"));
    SS_TRY(hip_status(ss::launch_gather(in->quats, keep_idx, n_keep, 4, (float*)out->quats, s),
                      "gather quats"));
    SS_TRY(hip_status(ss::launch_gather(in->opacity, keep_idx, n_keep, 1, (float*)out->opacity, s),
                      "gather opacity"));
    return hip_status(ss::launch_gather(in->sh, keep_idx, n_keep, 3 * in->sh_stride,
                                        (float*)out->sh, s),
                      "gather sh");
}

int ss_render_backward(const ss_camera* cam, const ss_gaussians* g, const ss_frame* f,
                       const ss_pairs* p, int32_t buf, const float* dl_drgb, const ss_grads* out,
                       const ss_stage_events* events, void* stream) {
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
        ss::launch_backward(*cam, *g, *f, p->values[buf], dl_drgb, *out,
                            events ? events->ev : nullptr, (hipStream_t)stream),
        "backward");
}

}  // extern "C"

"""CPU oracle for the Speedy-Splat forward rasterizer and its gradients.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
never imports, links or calls it, and it shares no code with the GPU library:
the only common dependency is the seeded input generator (``scenegen``), which
holds none of the method's arithmetic.

Layout:
  ref.c       plain C loops for every forward stage (FP64 geometry over FP32
              records, FP32 blend, FP64 brute force).  Built with gcc here.
  brute.py    plain definitions used as pins: the exact tile predicate TILE*
              (FP64 and exact-rational), dense ellipse sampling.
  grad.py     FP64 dense differentiable renderer (torch CPU) for gradients.

Functions whose result has no independent pin say "parity unpinned" in their
docstring.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

MODE_3SIGMA, MODE_SNUGBOX, MODE_ACCUTILE = 0, 1, 2
MODES = {"3sigma": MODE_3SIGMA, "snugbox": MODE_SNUGBOX, "accutile": MODE_ACCUTILE}
TILE = 16

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ref.c")
_LIB_PATH = os.path.join(_HERE, "_ref.so")
_lib = None
_lock = threading.Lock()

_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int


def build(force: bool = False) -> str:
    """Compile ref.c into _ref.so (plain gcc, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB_PATH)
            L.orc_sh_basis.argtypes = [ctypes.c_double] * 3 + [_f64p]
            L.orc_sh_basis.restype = None
            L.orc_tile_list.argtypes = [_f32p, _f32p, _int, _int, _int, _vp]
            L.orc_tile_list.restype = _i64
            L.orc_tile_rect.argtypes = [_f32p, _f32p, _int, _int, _int, _i32p]
            L.orc_tile_rect.restype = _int
            L.orc_preprocess.argtypes = [_f32p, _i64, _int, _int, _f32p, _f32p, _f32p, _f32p,
                                         _f32p, _int, _f32p, _f32p, _f32p, _u32p]
            L.orc_preprocess.restype = _i64
            L.orc_emit.argtypes = [_i64, _f32p, _f32p, _int, _int, _int, _u64p, _u32p]
            L.orc_emit.restype = _i64
            L.orc_sort.argtypes = [_i64, _u64p, _u32p]
            L.orc_sort.restype = None
            L.orc_ranges.argtypes = [_i64, _u64p, _i64, _u32p]
            L.orc_ranges.restype = None
            L.orc_blend.argtypes = [_f32p, _u32p, _u32p, _f32p, _f32p, _f32p, _i64, _vp,
                                    _f32p, _f32p, _u32p, _u32p, _u32p, _u8p]
            L.orc_blend.restype = None
            L.orc_brute_pixels.argtypes = [_f32p, _i64, _f32p, _f32p, _f32p, _i64p, _i64, _int,
                                           _i64, _i32p, _f64p, _u8p]
            L.orc_brute_pixels.restype = None
            L.orc_extent.argtypes = [_f32p, _f32p, _int, _f64p]
            L.orc_extent.restype = _int
            _lib = L
    return _lib


def mode_id(mode) -> int:
    return MODES[mode] if isinstance(mode, str) else int(mode)


def camera_pack(cam) -> np.ndarray:
    """24-float camera block understood by ref.c (width, height, fx, fy, cx, cy,
    R row-major, t, near, background)."""
    p = np.zeros(24, dtype=np.float32)
    p[0], p[1] = cam.width, cam.height
    p[2:6] = (cam.fx, cam.fy, cam.cx, cam.cy)
    p[6:15] = np.asarray(cam.R, dtype=np.float32).reshape(9)
    p[15:18] = np.asarray(cam.t, dtype=np.float32).reshape(3)
    p[18] = cam.near
    p[19:22] = cam.bg
    return p


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ------------------------------------------------------------------ stages

class Records:
    """FP32 per-Gaussian records: geom (u, v, depth, t), conic (a, b, c, sigma),
    rgb (r, g, b, 0) and the tile count for the mode."""

    def __init__(self, geom, conic, rgb, counts, mode, visible):
        self.geom, self.conic, self.rgb, self.counts = geom, conic, rgb, counts
        self.mode, self.visible = mode, visible

    @property
    def n(self):
        return self.geom.shape[0]


def sh_basis(direction) -> np.ndarray:
    """Real SH basis (16 values, degree <= 3) at a unit direction."""
    out = np.zeros(16, dtype=np.float64)
    x, y, z = (float(c) for c in direction)
    lib().orc_sh_basis(x, y, z, out)
    return out


def preprocess(scene, cam, mode) -> Records:
    """Per-Gaussian records and tile counts (camera space, projection, Sigma_3D,
    EWA with +0.3 dilation, conic, t = 2 log(255 sigma), SH colour, then the
    mode's tile count on the stored record)."""
    m = mode_id(mode)
    n = scene.n
    geom = np.zeros((n, 4), np.float32)
    conic = np.zeros((n, 4), np.float32)
    rgb = np.zeros((n, 4), np.float32)
    counts = np.zeros(n, np.uint32)
    sh = _c(scene.sh, np.float32)
    stride = sh.shape[1]
    vis = lib().orc_preprocess(camera_pack(cam), n, int(scene.sh_degree), stride,
                               _c(scene.means, np.float32), _c(scene.scales, np.float32),
                               _c(scene.quats, np.float32), _c(scene.opacity, np.float32),
                               sh.reshape(-1), m, geom, conic, rgb, counts)
    return Records(geom, conic, rgb, counts, m, int(vis))


def tile_list(geom_i, conic_i, mode, tiles_x, tiles_y) -> np.ndarray:
    """Tile ids of one record in emission order."""
    g = _c(geom_i, np.float32).reshape(4)
    q = _c(conic_i, np.float32).reshape(4)
    L = lib()
    cnt = L.orc_tile_list(g, q, mode_id(mode), tiles_x, tiles_y, None)
    out = np.zeros(max(cnt, 1), np.uint32)
    L.orc_tile_list(g, q, mode_id(mode), tiles_x, tiles_y, out.ctypes.data)
    return out[:cnt]


def tile_rect(geom_i, conic_i, mode, tiles_x, tiles_y):
    """Inclusive tile rectangle (x0, y0, x1, y1) of one record; None when empty."""
    r = np.zeros(4, np.int32)
    ok = lib().orc_tile_rect(_c(geom_i, np.float32).reshape(4), _c(conic_i, np.float32).reshape(4),
                             mode_id(mode), tiles_x, tiles_y, r)
    return tuple(int(x) for x in r) if ok else None


def extent(geom_i, conic_i, mode):
    """Pixel-space box (x0, x1, y0, y1) of one record: the 3-sigma square or the
    SnugBox box; None when the record has no extent."""
    out = np.zeros(4, np.float64)
    ok = lib().orc_extent(_c(geom_i, np.float32).reshape(4), _c(conic_i, np.float32).reshape(4),
                          mode_id(mode), out)
    return tuple(out) if ok else None


def emit(rec: Records, cam):
    """Unsorted (key, value) pairs in emission order."""
    p = int(rec.counts.astype(np.uint64).sum())
    keys = np.zeros(max(p, 1), np.uint64)
    vals = np.zeros(max(p, 1), np.uint32)
    got = lib().orc_emit(rec.n, rec.geom, rec.conic, rec.mode, cam.tiles_x, cam.tiles_y, keys, vals)
    assert got == p, (got, p)
    return keys[:p], vals[:p]


def sort_pairs(keys, values):
    k = keys.copy()
    v = values.copy()
    if len(k):
        lib().orc_sort(len(k), k, v)
    return k, v


def tile_ranges(keys, n_tiles) -> np.ndarray:
    r = np.zeros((n_tiles, 2), np.uint32)
    k = keys if len(keys) else np.zeros(1, np.uint64)
    lib().orc_ranges(len(keys), _c(k, np.uint64), n_tiles, r)
    return r


def blend(cam, ranges, values, rec: Records, tiles=None):
    """FP32 tiled blend.  Returns (img[3,H,W], T_final[H,W], n_last[H,W],
    ambiguous[H,W], n_eval[H,W], n_contrib[H,W]).  With ``tiles`` given, only
    those tile ids are written.  n_eval counts the list entries a pixel
    evaluated before it stopped, n_contrib the Gaussians blended into it."""
    H, W = cam.height, cam.width
    ne = np.zeros((H, W), np.uint32)
    nc = np.zeros((H, W), np.uint32)
    img = np.zeros((3, H, W), np.float32)
    tf = np.zeros((H, W), np.float32)
    nl = np.zeros((H, W), np.uint32)
    amb = np.zeros((H, W), np.uint8)
    vals = values if len(values) else np.zeros(1, np.uint32)
    if tiles is None:
        lib().orc_blend(camera_pack(cam), _c(ranges, np.uint32).reshape(-1), _c(vals, np.uint32),
                        rec.geom, rec.conic, rec.rgb, -1, None, img, tf, nl, ne, nc, amb)
    else:
        tl = _c(tiles, np.int32)
        lib().orc_blend(camera_pack(cam), _c(ranges, np.uint32).reshape(-1), _c(vals, np.uint32),
                        rec.geom, rec.conic, rec.rgb, len(tl), tl.ctypes.data, img, tf, nl, ne,
                        nc, amb)
    return img, tf, nl, amb.astype(bool), ne, nc


def depth_order(rec: Records) -> np.ndarray:
    """Global front-to-back order of the surviving records: by depth bits, then index."""
    alive = np.nonzero((rec.conic[:, 0] != 0) | (rec.conic[:, 1] != 0) | (rec.conic[:, 2] != 0))[0]
    bits = rec.geom[alive, 2].view(np.uint32)
    return alive[np.lexsort((alive, bits))].astype(np.int64)


def brute_pixels(cam, rec: Records, pixels, rect_mode=None):
    """FP64 brute force over every record for the given (px, py) pixels.
    rect_mode=None is B-infinity; rect_mode=MODE_3SIGMA restricts each record to
    its 3-sigma tile rectangle.  Returns (rgb[k,3], ambiguous[k])."""
    pix = _c(np.asarray(pixels).reshape(-1, 2), np.int32)
    order = depth_order(rec)
    out = np.zeros((len(pix), 3), np.float64)
    amb = np.zeros(len(pix), np.uint8)
    lib().orc_brute_pixels(camera_pack(cam), rec.n, rec.geom, rec.conic, rec.rgb,
                           order if len(order) else np.zeros(1, np.int64), len(order),
                           -1 if rect_mode is None else mode_id(rect_mode),
                           len(pix), pix.reshape(-1), out.reshape(-1), amb)
    return out, amb.astype(bool)


def all_pixels(cam) -> np.ndarray:
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    return np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.int32)


class Frame:
    """Every intermediate of one oracle render."""

    def __init__(self, **kw):
        self.__dict__.update(kw)


def render(scene, cam, mode, blend_tiles="all") -> Frame:
    """Whole forward pipeline: records, counts, offsets, P, unsorted and sorted
    pairs, tile ranges and the blended image.  ``blend_tiles`` = "all", None
    (skip the blend) or a list of tile ids."""
    rec = preprocess(scene, cam, mode)
    offsets = np.cumsum(rec.counts.astype(np.uint64))
    keys, vals = emit(rec, cam)
    skeys, svals = sort_pairs(keys, vals)
    n_tiles = cam.tiles_x * cam.tiles_y
    ranges = tile_ranges(skeys, n_tiles)
    img = tf = nl = amb = ne = nc = None
    if blend_tiles is not None:
        img, tf, nl, amb, ne, nc = blend(cam, ranges, svals, rec,
                                         None if isinstance(blend_tiles, str) else blend_tiles)
    return Frame(records=rec, offsets=offsets, n_pairs=int(offsets[-1]) if len(offsets) else 0,
                 keys=keys, values=vals, sorted_keys=skeys, sorted_values=svals,
                 ranges=ranges, image=img, t_final=tf, n_last=nl, ambiguous=amb,
                 n_eval=ne, n_contrib=nc)

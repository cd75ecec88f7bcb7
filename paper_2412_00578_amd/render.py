"""Python face of the rasterizer: device buffers from torch, work in the library.

    import paper_2412_00578_amd as ss
    g = ss.Gaussians.from_arrays(means, scales, quats, opacity, sh, sh_degree, device="cuda")
    r = ss.Renderer()
    image = r.render(g, camera, "accutile")          # [3, H, W] float32 on the device

torch allocates every buffer (the library allocates nothing) and supplies the
stream; each call below is one or more C-ABI calls on the current stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import check, lib, make_camera, mode_id


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Gaussians:
    """Device-resident Gaussian parameters (the C ABI's ss_gaussians)."""

    def __init__(self, means, scales, quats, opacity, sh, sh_degree: int):
        self.means = means.contiguous()
        self.scales = scales.contiguous()
        self.quats = quats.contiguous()
        self.opacity = opacity.contiguous().reshape(-1)
        self.sh = sh.contiguous()
        self.sh_degree = int(sh_degree)
        for t in (self.means, self.scales, self.quats, self.opacity, self.sh):
            if t.dtype != torch.float32:
                raise TypeError("Gaussian parameters must be float32")

    @classmethod
    def from_arrays(cls, means, scales, quats, opacity, sh, sh_degree, device="cuda"):
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=device)
        return cls(f(means), f(scales), f(quats), f(opacity), f(sh), sh_degree)

    @classmethod
    def from_scene(cls, scene, device="cuda"):
        return cls.from_arrays(scene.means, scene.scales, scene.quats, scene.opacity, scene.sh,
                               scene.sh_degree, device)

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def device(self):
        return self.means.device

    @property
    def nbytes(self) -> int:
        return sum(t.numel() * 4 for t in (self.means, self.scales, self.quats, self.opacity,
                                           self.sh))

    def struct(self) -> _lib.SSGaussians:
        s = _lib.SSGaussians()
        s.n = self.n
        s.sh_degree = self.sh_degree
        s.sh_stride = int(self.sh.shape[1]) if self.sh.dim() == 3 else 1
        s.means, s.scales, s.quats = (self.means.data_ptr(), self.scales.data_ptr(),
                                      self.quats.data_ptr())
        s.opacity, s.sh = self.opacity.data_ptr(), self.sh.data_ptr()
        return s


class Frame:
    """Per-frame buffers (ss_frame) for n Gaussians at width x height."""

    def __init__(self, n: int, width: int, height: int, device, stats: bool = True):
        info = _lib.SSFrameInfo()
        check(lib().ss_frame_sizes(n, width, height, ctypes.byref(info)), "ss_frame_sizes")
        self.info = info
        self.n, self.width, self.height = n, width, height
        dev = torch.device(device)
        # geom and conic interleaved: one [n, 8] buffer, two [n, 4] views
        self.records = torch.empty((n, 8), dtype=torch.float32, device=dev)
        self.geom, self.conic = self.records[:, :4], self.records[:, 4:]
        self.rgb = torch.empty((n, 4), dtype=torch.float32, device=dev)
        self.counts = torch.empty(n, dtype=torch.int32, device=dev)
        self.depth_keys = torch.empty(2 * n, dtype=torch.int32, device=dev)
        self.order = torch.empty(2 * n, dtype=torch.int32, device=dev)
        self.order_counts = torch.empty(n, dtype=torch.int32, device=dev)
        self.order_tmp = torch.empty(int(info.order_tmp_words), dtype=torch.int32, device=dev)
        self.tile_sets = torch.empty((n, 4), dtype=torch.int32, device=dev)
        self.offsets = torch.empty(n, dtype=torch.int32, device=dev)
        self.scan_tmp = torch.zeros(int(info.scan_tmp_words), dtype=torch.int64, device=dev)
        self.totals = torch.zeros(2, dtype=torch.int64, device=dev)
        self.ranges = torch.empty((info.n_tiles, 2), dtype=torch.int32, device=dev)
        self.t_final = torch.empty((height, width), dtype=torch.float32, device=dev)
        self.n_last = torch.empty((height, width), dtype=torch.int32, device=dev)
        # per-pixel counts of evaluated list entries and of blended Gaussians
        # (statistics; NULL skips them)
        self.n_eval = torch.empty((height, width), dtype=torch.int32, device=dev) if stats else None
        self.n_contrib = (torch.empty((height, width), dtype=torch.int32, device=dev)
                          if stats else None)
        self.emit_tmp = torch.empty(int(info.emit_tmp_words), dtype=torch.int32, device=dev)
        self.table = torch.empty(int(info.table_bytes), dtype=torch.uint8, device=dev)

    def struct(self) -> _lib.SSFrame:
        f = _lib.SSFrame()
        for name in ("geom", "conic", "rgb", "counts", "depth_keys", "order", "order_counts",
                     "order_tmp", "tile_sets", "offsets", "scan_tmp", "totals", "ranges",
                     "t_final", "n_last", "n_eval", "n_contrib", "emit_tmp", "table"):
            t = getattr(self, name)
            setattr(f, name, t.data_ptr() if t is not None else None)
        return f

    def fits(self, n, width, height, stats=True) -> bool:
        return (self.n == n and self.width == width and self.height == height
                and (self.n_eval is not None) == stats)


class Pairs:
    """Pair workspace (ss_pairs): two tile-key/value buffers and sort scratch."""

    def __init__(self, capacity: int, device):
        dev = torch.device(device)
        cap = max(int(capacity), 1)
        self.capacity = cap
        self.keys = [torch.empty(cap, dtype=torch.int32, device=dev) for _ in range(2)]
        self.values = [torch.empty(cap, dtype=torch.int32, device=dev) for _ in range(2)]
        w = ctypes.c_int64()
        check(lib().ss_sort_tmp_words(cap, ctypes.byref(w)), "ss_sort_tmp_words")
        self.sort_tmp = torch.empty(int(w.value), dtype=torch.int32, device=dev)

    def struct(self) -> _lib.SSPairs:
        p = _lib.SSPairs()
        p.capacity = self.capacity
        p.keys[0], p.keys[1] = self.keys[0].data_ptr(), self.keys[1].data_ptr()
        p.values[0], p.values[1] = self.values[0].data_ptr(), self.values[1].data_ptr()
        p.sort_tmp = self.sort_tmp.data_ptr()
        return p


# "ranges" covers the tile ranges and the blend's tile work order, so that
# "blend" is the blend kernel alone
STAGES = ("preprocess", "readback", "depth_order", "scan", "emit", "sort", "ranges", "blend")


class BackwardEvents:
    """Four timing events ss_render_backward records: start, after zeroing the
    accumulators, after the blend adjoint, after the preprocess adjoint."""

    def __init__(self, device):
        self.events = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        s = torch.cuda.current_stream(device)
        for e in self.events:  # creates the underlying hipEvent_t
            e.record(s)
        s.synchronize()

    def struct(self) -> _lib.SSStageEvents:
        st = _lib.SSStageEvents()
        for k, e in enumerate(self.events):
            st.ev[k] = e.cuda_event
        return st

    def ms(self) -> dict:
        e = self.events
        return {"zero": e[0].elapsed_time(e[1]), "blend_bwd": e[1].elapsed_time(e[2]),
                "preprocess_bwd": e[2].elapsed_time(e[3])}


class StageEvents:
    """Nine timing events recorded by the library at stage boundaries."""

    def __init__(self, device):
        self.events = [torch.cuda.Event(enable_timing=True) for _ in range(len(STAGES) + 1)]
        s = torch.cuda.current_stream(device)
        for e in self.events:  # creates the underlying hipEvent_t
            e.record(s)
        s.synchronize()

    def struct(self) -> _lib.SSStageEvents:
        st = _lib.SSStageEvents()
        for k, e in enumerate(self.events):
            st.ev[k] = e.cuda_event
        return st

    def stage_ms(self) -> dict:
        """Per-stage milliseconds of the last recorded frame (after a sync)."""
        ev = self.events
        return {name: ev[k].elapsed_time(ev[k + 1]) for k, name in enumerate(STAGES)}

    def frame_ms(self) -> float:
        return self.events[0].elapsed_time(self.events[len(STAGES)])


@dataclass
class RenderOutput:
    image: torch.Tensor      # [3, H, W]
    n_pairs: int
    n_visible: int           # Gaussians with at least one tile
    frame: Frame
    pairs: Pairs
    buf: int                 # pair buffer holding the sorted pairs


@dataclass
class NoSyncRender:
    """A frame queued by Renderer.render_nosync."""
    image: torch.Tensor
    frame: "Frame"
    pairs: "Pairs"
    buf: int
    counts: torch.Tensor     # pinned [2]: P, Gaussians with tiles (valid after the sync)
    capacity: int

    @property
    def n_pairs(self) -> int:
        return int(self.counts[0])

    def ok(self) -> bool:
        """True when the pair workspace held the frame (call after the sync)."""
        p = int(self.counts[0])
        if p < 0:
            raise RuntimeError("frame counts not copied yet: synchronise the stream first")
        return p <= self.capacity


class Renderer:
    """Owns reusable frame and pair buffers; grows them on demand."""

    def __init__(self, device="cuda", growth: float = 1.25, stats: bool = False):
        """stats=True also records, per pixel, how many list entries it evaluated
        (Frame.n_eval)."""
        self.device = torch.device(device)
        self.growth = growth
        self.stats = stats
        self._frame: Frame | None = None
        self._pairs: Pairs | None = None
        self._ring: list = [None] * self.RING    # frames of render_many
        self._host_p: torch.Tensor | None = None
        self._side = None                        # side streams of render_many
        self._max_pairs = 0                      # largest pair count seen (sizes render_nosync)
        self._nosync_counts: torch.Tensor | None = None
        self._nosync_next = 0

    def frame_for(self, n, width, height) -> Frame:
        if self._frame is None or not self._frame.fits(n, width, height, self.stats):
            self._frame = None
            self._frame = Frame(n, width, height, self.device, self.stats)
        return self._frame

    def pairs_for(self, n_pairs) -> Pairs:
        if self._pairs is None or self._pairs.capacity < n_pairs:
            self._pairs = None
            self._pairs = Pairs(int(max(n_pairs, 1) * self.growth) + 1024, self.device)
        return self._pairs

    # ---- whole forward -------------------------------------------------------
    def render(self, g: Gaussians, cam, mode="accutile", out: torch.Tensor | None = None,
               full: bool = False, events: "StageEvents | None" = None):
        """Forward render.  Returns the image [3,H,W] (or a RenderOutput if full).
        ``events`` (a StageEvents) records per-stage timing on the stream."""
        m = mode_id(mode)
        c = make_camera(cam)
        frame = self.frame_for(g.n, c.width, c.height)
        if out is None:
            out = torch.empty((3, c.height, c.width), dtype=torch.float32, device=self.device)
        gs, fs = g.struct(), frame.struct()
        stream = _stream(self.device)
        counts = _lib.SSFrameCounts()
        ev = events.struct() if events is not None else None
        evp = ctypes.byref(ev) if ev is not None else None
        check(lib().ss_forward_begin(ctypes.byref(c), ctypes.byref(gs), m, ctypes.byref(fs),
                                     ctypes.byref(counts), evp, stream), "ss_forward_begin")
        self._max_pairs = max(self._max_pairs, int(counts.n_pairs))
        pairs = self.pairs_for(counts.n_pairs)
        ps = pairs.struct()
        buf = ctypes.c_int32()
        check(lib().ss_forward_finish(ctypes.byref(c), g.n, m, ctypes.byref(fs), ctypes.byref(ps),
                                      ctypes.byref(counts), _ptr(out), ctypes.byref(buf), evp,
                                      stream), "ss_forward_finish")
        if full:
            return RenderOutput(out, int(counts.n_pairs), int(counts.n_visible), frame, pairs,
                                int(buf.value))
        return out

    NOSYNC_SLOTS = 256   # frame-count slots of render_nosync (frames in flight)

    def render_nosync(self, g: Gaussians, cam, mode="accutile", out: torch.Tensor | None = None,
                      events: "StageEvents | None" = None) -> "NoSyncRender":
        """Forward render with no host synchronisation (ss_render_nosync): every
        stage is queued at once, the later ones reading the frame counts on the
        device, so frames can be queued back to back without the GPU waiting for
        a read-back.  The pair workspace is the renderer's, sized for the
        largest frame it has seen (with growth headroom).  The frame counts land
        in a pinned slot; once the stream has been synchronised, the returned
        object's ok() tells whether the workspace held the frame (if not, the
        image is the background alone: render() the frame instead, which also
        grows the workspace).  At most NOSYNC_SLOTS frames may be checked late."""
        m = mode_id(mode)
        c = make_camera(cam)
        frame = self.frame_for(g.n, c.width, c.height)
        if out is None:
            out = torch.empty((3, c.height, c.width), dtype=torch.float32, device=self.device)
        if self._nosync_counts is None:
            self._nosync_counts = torch.zeros((self.NOSYNC_SLOTS, 2), dtype=torch.int64,
                                              pin_memory=True)
        slot = self._nosync_next % self.NOSYNC_SLOTS
        self._nosync_next += 1
        host = self._nosync_counts[slot]
        host.fill_(-1)
        pairs = self.pairs_for(max(self._max_pairs, 1))
        gs, fs, ps = g.struct(), frame.struct(), pairs.struct()
        buf = ctypes.c_int32()
        ev = events.struct() if events is not None else None
        check(lib().ss_render_nosync(ctypes.byref(c), ctypes.byref(gs), m, ctypes.byref(fs),
                                     ctypes.byref(ps), _ptr(out), ctypes.c_void_p(host.data_ptr()),
                                     ctypes.byref(buf), ctypes.byref(ev) if ev is not None else None,
                                     _stream(self.device)), "ss_render_nosync")
        return NoSyncRender(out, frame, pairs, int(buf.value), host, pairs.capacity)

    def render_band(self, g: Gaussians, cam, mode, tile_row0: int, tile_rows: int,
                    out: torch.Tensor | None = None, full: bool = False,
                    events: "StageEvents | None" = None):
        """Forward render of the band of tile rows [tile_row0, tile_row0 +
        tile_rows) of the camera's image (ss_render_band): every Gaussian is
        preprocessed, only the band's tiles are rendered.  Returns the band's
        image [3, band_height, W] (or a RenderOutput with the band's frame and
        pairs if full)."""
        m = mode_id(mode)
        c = make_camera(cam)
        y_end = min(c.height, 16 * (tile_row0 + tile_rows))
        bh = max(y_end - 16 * tile_row0, 1)
        frame = self.frame_for(g.n, c.width, bh)
        if out is None:
            out = torch.empty((3, bh, c.width), dtype=torch.float32, device=self.device)
        gs, fs = g.struct(), frame.struct()
        counts = _lib.SSFrameCounts()
        buf = ctypes.c_int32()
        ev = events.struct() if events is not None else None
        evp = ctypes.byref(ev) if ev is not None else None
        for attempt in range(2):
            pairs = self.pairs_for(counts.n_pairs)
            ps = pairs.struct()
            st = lib().ss_render_band(ctypes.byref(c), ctypes.byref(gs), m, int(tile_row0),
                                      int(tile_rows), ctypes.byref(fs), ctypes.byref(ps),
                                      _ptr(out), ctypes.byref(counts), ctypes.byref(buf), evp,
                                      _stream(self.device))
            if st != _lib.SS_ERR_WORKSPACE or attempt == 1:
                check(st, "ss_render_band")
                break
        if full:
            return RenderOutput(out, int(counts.n_pairs), int(counts.n_visible), frame, pairs,
                                int(buf.value))
        return out

    RING = 3   # frame buffers of render_many

    def render_many(self, g: Gaussians, cams, mode="accutile", outs=None) -> list:
        """Renders one frame per camera as a pipeline over three HIP streams and
        three frame buffers: a side stream runs frame k + 2's preprocess and
        frame-count read-back, a second one frame k + 1's depth order and scan,
        and the current stream frame k's emit, sort, ranges and blend.  The
        preprocess is bound by FP64 work and memory latency, the depth order by
        latency, the blend by the FP32 vector ALUs, so they overlap on the GPU.
        The counts come back by asynchronous copies; the host waits for a
        frame's counts (it sizes the depth order and the pair buffer with them)
        only after it has queued the back half of the frame before.  Every
        frame is rendered completely and identically to render(); the images
        are valid once the current stream syncs."""
        m = mode_id(mode)
        cs = [make_camera(c) for c in cams]
        if outs is None:
            outs = [torch.empty((3, c.height, c.width), dtype=torch.float32, device=self.device)
                    for c in cs]
        if not cs:
            return outs
        main = torch.cuda.current_stream(self.device)
        if self._side is None:            # default priority, like every stream here
            self._side = (torch.cuda.Stream(self.device), torch.cuda.Stream(self.device))
        side, mid = self._side
        side.wait_stream(main)             # earlier work on the ring buffers is done
        mid.wait_stream(main)
        smain = ctypes.c_void_p(main.cuda_stream)
        sside = ctypes.c_void_p(side.cuda_stream)
        smid = ctypes.c_void_p(mid.cuda_stream)
        gs = g.struct()
        R = self.RING
        if self._host_p is None:           # one ss_frame_counts per frame buffer
            self._host_p = torch.zeros((R, 2), dtype=torch.int64, pin_memory=True)
        host = self._host_p
        ready = [torch.cuda.Event() for _ in range(R)]   # counts copied (side stream)
        front = [torch.cuda.Event() for _ in range(R)]   # depth order and scan done (mid)
        free = [torch.cuda.Event() for _ in range(R)]    # frame buffer released (main)
        fss = [None] * R
        counts = [None] * len(cs)

        def preprocess(k):
            r = k % R
            if k >= R:
                side.wait_event(free[r])
            f = self._ring[r]
            if f is None or not f.fits(g.n, cs[k].width, cs[k].height, self.stats):
                side.synchronize()         # a resize: nothing may still use the old buffers
                mid.synchronize()
                main.synchronize()
                self._ring[r] = None
                self._ring[r] = f = Frame(g.n, cs[k].width, cs[k].height, self.device,
                                          self.stats)
            fss[r] = f.struct()
            check(lib().ss_forward_begin_async(ctypes.byref(cs[k]), ctypes.byref(gs), m,
                                               ctypes.byref(fss[r]),
                                               ctypes.c_void_p(host.data_ptr() + 16 * r), None,
                                               sside), "ss_forward_begin_async")
            ready[r].record(side)

        def order(k):                      # waits for frame k's counts
            r = k % R
            ready[r].synchronize()
            c = counts[k] = _lib.SSFrameCounts(int(host[r, 0]), int(host[r, 1]))
            if c.n_pairs >= 0xffffffff:
                raise RuntimeError(f"{c.n_pairs} pairs do not fit 32-bit offsets")
            mid.wait_event(ready[r])
            check(lib().ss_depth_order(g.n, c.n_visible, ctypes.byref(fss[r]), smid),
                  "ss_depth_order")
            check(lib().ss_scan(c.n_visible, ctypes.byref(fss[r]), smid), "ss_scan")
            front[r].record(mid)

        def back(k):
            r = k % R
            c = counts[k]
            main.wait_event(front[r])
            pairs = self.pairs_for(c.n_pairs)
            ps = pairs.struct()
            buf = ctypes.c_int32()
            check(lib().ss_forward_back(ctypes.byref(cs[k]), g.n, m, ctypes.byref(fss[r]),
                                        ctypes.byref(ps), ctypes.byref(c), _ptr(outs[k]),
                                        ctypes.byref(buf), None, smain), "ss_forward_back")
            free[r].record(main)

        # preprocess k + 2 is queued before the host waits for frame k + 1's
        # counts, so the side stream never idles while the host waits
        preprocess(0)
        if len(cs) > 1:
            preprocess(1)
        order(0)
        for k in range(len(cs)):
            back(k)
            if k + 2 < len(cs):
                preprocess(k + 2)
            if k + 1 < len(cs):
                order(k + 1)
        return outs

    # ---- single stages (for tests and profiling) ---------------------------
    def preprocess(self, g: Gaussians, cam, mode) -> Frame:
        c = make_camera(cam)
        frame = self.frame_for(g.n, c.width, c.height)
        gs, fs = g.struct(), frame.struct()
        check(lib().ss_preprocess(ctypes.byref(c), ctypes.byref(gs), mode_id(mode),
                                  ctypes.byref(fs), _stream(self.device)), "ss_preprocess")
        return frame

    def counts(self, frame: Frame) -> tuple:
        """(P, n_visible) the preprocess stage accumulated (synchronises)."""
        torch.cuda.current_stream(self.device).synchronize()
        t = frame.totals.cpu()
        return int(t[0]), int(t[1])

    def depth_order(self, frame: Frame, n_visible: int) -> torch.Tensor:
        """Stage 2a; returns frame.order[:n_visible] (Gaussians with tiles by
        depth, then index)."""
        fs = frame.struct()
        check(lib().ss_depth_order(frame.n, n_visible, ctypes.byref(fs), _stream(self.device)),
              "ss_depth_order")
        return frame.order[:n_visible]

    def scan(self, frame: Frame, n_visible: int) -> int:
        fs = frame.struct()
        check(lib().ss_scan(n_visible, ctypes.byref(fs), _stream(self.device)), "ss_scan")
        torch.cuda.current_stream(self.device).synchronize()
        return int(frame.scan_tmp[0].item())

    def emit(self, cam, frame: Frame, mode, n_visible: int, n_pairs: int, buf: int = 0) -> Pairs:
        c = make_camera(cam)
        pairs = self.pairs_for(n_pairs)
        fs, ps = frame.struct(), pairs.struct()
        check(lib().ss_emit(ctypes.byref(c), frame.n, n_visible, mode_id(mode), ctypes.byref(fs),
                            ctypes.byref(ps), buf, n_pairs, _stream(self.device)), "ss_emit")
        return pairs

    def sort(self, cam, pairs: Pairs, n_pairs: int, buf: int = 0) -> int:
        c = make_camera(cam)
        ps = pairs.struct()
        ob = ctypes.c_int32()
        check(lib().ss_sort(ctypes.byref(c), ctypes.byref(ps), buf, n_pairs, ctypes.byref(ob),
                            _stream(self.device)), "ss_sort")
        return int(ob.value)

    def ranges(self, cam, frame: Frame, pairs: Pairs, n_pairs: int, buf: int):
        c = make_camera(cam)
        fs, ps = frame.struct(), pairs.struct()
        check(lib().ss_ranges(ctypes.byref(c), ctypes.byref(fs), ctypes.byref(ps), buf, n_pairs,
                              _stream(self.device)), "ss_ranges")

    def blend(self, cam, frame: Frame, pairs: Pairs, buf: int, out=None) -> torch.Tensor:
        c = make_camera(cam)
        if out is None:
            out = torch.empty((3, c.height, c.width), dtype=torch.float32, device=self.device)
        fs, ps = frame.struct(), pairs.struct()
        check(lib().ss_blend(ctypes.byref(c), ctypes.byref(fs), ctypes.byref(ps), buf, _ptr(out),
                             _stream(self.device)), "ss_blend")
        return out


# ---------------------------------------------------------------- gradients

@dataclass
class Grads:
    means: torch.Tensor
    scales: torch.Tensor
    quats: torch.Tensor
    opacity: torch.Tensor
    sh: torch.Tensor
    g2d: torch.Tensor        # [n, 12] screen-space gradients
    #                          (u, v, -, -, a, b, c, sigma, r, g, b, -)
    score: torch.Tensor | None


def backward(g: Gaussians, cam, out: RenderOutput, dl_drgb: torch.Tensor,
             want_score: bool = False, sh_out: torch.Tensor | None = None,
             events: "BackwardEvents | None" = None) -> Grads:
    """Adjoint of a forward render `out` (from Renderer.render(..., full=True)).
    sh_out: optional caller-owned [n, K, 3] float32 buffer (any 4-byte
    alignment) that receives dL/dh.  events: optional BackwardEvents that time
    the blend adjoint and the preprocess adjoint."""
    c = make_camera(cam)
    dev = g.device
    dl = dl_drgb.contiguous().to(torch.float32)
    if sh_out is not None and (tuple(sh_out.shape) != tuple(g.sh.shape) or
                               not sh_out.is_contiguous() or sh_out.dtype != torch.float32):
        raise ValueError("sh_out must be a contiguous float32 tensor shaped like the SH")
    if tuple(dl.shape) != (3, c.height, c.width):
        raise ValueError(f"dl_drgb must be [3, {c.height}, {c.width}]")
    n = g.n
    gr = Grads(torch.empty_like(g.means), torch.empty_like(g.scales), torch.empty_like(g.quats),
               torch.empty_like(g.opacity), torch.empty_like(g.sh) if sh_out is None else sh_out,
               torch.empty((n, 12), dtype=torch.float32, device=dev),
               torch.empty(n, dtype=torch.float32, device=dev) if want_score else None)
    st = _lib.SSGrads()
    st.means, st.scales, st.quats = gr.means.data_ptr(), gr.scales.data_ptr(), gr.quats.data_ptr()
    st.opacity, st.sh, st.g2d = gr.opacity.data_ptr(), gr.sh.data_ptr(), gr.g2d.data_ptr()
    st.score = gr.score.data_ptr() if want_score else None
    gs, fs, ps = g.struct(), out.frame.struct(), out.pairs.struct()
    check(lib().ss_render_backward(ctypes.byref(c), ctypes.byref(gs), ctypes.byref(fs),
                                   ctypes.byref(ps), out.buf, _ptr(dl), ctypes.byref(st),
                                   ctypes.byref(events.struct()) if events else None,
                                   _stream(dev)), "ss_render_backward")
    return gr


class _Rasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, scales, quats, opacity, sh, cam, mode, sh_degree):
        g = Gaussians(means.detach(), scales.detach(), quats.detach(), opacity.detach(),
                      sh.detach(), sh_degree)
        r = Renderer(means.device)   # buffers owned by this call, kept for its backward
        out = r.render(g, cam, mode, full=True)
        ctx.state = (g, cam, out)
        return out.image

    @staticmethod
    def backward(ctx, grad_img):
        g, cam, out = ctx.state
        gr = backward(g, cam, out, grad_img)
        ctx.state = None
        return gr.means, gr.scales, gr.quats, gr.opacity, gr.sh, None, None, None


def render(means, scales, quats, opacity, sh, camera, mode="accutile", sh_degree=None):
    """Differentiable forward render (a torch.autograd.Function).

    means [N,3], scales [N,3] (linear, > 0), quats [N,4] (w, x, y, z),
    opacity [N] in (0, 1], sh [N, K, 3]; all float32 on the GPU.  Apply the
    activations (e.g. exp of log-scales, sigmoid of logits) in torch before the
    call.  Returns the image [3, H, W]."""
    deg = int(round(sh.shape[1] ** 0.5)) - 1 if sh_degree is None else int(sh_degree)
    return _Rasterize.apply(means, scales, quats, opacity.reshape(-1), sh, camera, mode, deg)


def pruning_score(g: Gaussians, cam, mode="accutile") -> torch.Tensor:
    """Per-Gaussian efficient pruning score: sum over pixels and colour channels
    of (dC/dg_i)^2, where g_i is the value of Gaussian i's projected 2D
    Gaussian at the pixel.  One forward and one adjoint pass."""
    r = Renderer(g.device)
    out = r.render(g, cam, mode, full=True)
    dl = torch.zeros((3, out.image.shape[1], out.image.shape[2]), dtype=torch.float32,
                     device=g.device)
    return backward(g, cam, out, dl, want_score=True).score


# ---------------------------------------------------------------- batches

class BatchFrame:
    """Frame buffers (ss_frame) of a batch: all items' records, tiles and pixels."""

    def __init__(self, info: _lib.SSBatchInfo, n_items: int, device, stats: bool = False):
        dev = torch.device(device)
        ns, npx = int(info.n_slots), int(info.n_pixels)
        self.info = info
        self.records = torch.empty((ns, 8), dtype=torch.float32, device=dev)
        self.geom, self.conic = self.records[:, :4], self.records[:, 4:]
        self.rgb = torch.empty((ns, 4), dtype=torch.float32, device=dev)
        self.counts = torch.empty(ns, dtype=torch.int32, device=dev)
        self.depth_keys = torch.empty(2 * ns, dtype=torch.int32, device=dev)
        self.order = torch.empty(2 * ns, dtype=torch.int32, device=dev)
        self.order_counts = torch.empty(ns, dtype=torch.int32, device=dev)
        self.order_tmp = torch.empty(int(info.order_tmp_words), dtype=torch.int32, device=dev)
        self.tile_sets = torch.empty((ns, 4), dtype=torch.int32, device=dev)
        self.offsets = torch.empty(ns, dtype=torch.int32, device=dev)
        self.scan_tmp = torch.zeros(int(info.scan_tmp_words), dtype=torch.int64, device=dev)
        self.totals = torch.zeros(2, dtype=torch.int64, device=dev)
        self.ranges = torch.empty((max(int(info.n_tiles), 1), 2), dtype=torch.int32, device=dev)
        self.t_final = torch.empty(max(npx, 1), dtype=torch.float32, device=dev)
        self.n_last = torch.empty(max(npx, 1), dtype=torch.int32, device=dev)
        self.n_eval = torch.empty(max(npx, 1), dtype=torch.int32, device=dev) if stats else None
        self.n_contrib = (torch.empty(max(npx, 1), dtype=torch.int32, device=dev)
                          if stats else None)
        self.emit_tmp = torch.empty(int(info.emit_tmp_words), dtype=torch.int32, device=dev)
        self.table = torch.empty(int(info.table_bytes), dtype=torch.uint8, device=dev)

    struct = Frame.struct

    @property
    def nbytes(self) -> int:
        return sum(t.numel() * t.element_size() for t in
                   (self.geom, self.conic, self.rgb, self.counts, self.depth_keys, self.order,
                    self.order_counts, self.order_tmp, self.tile_sets, self.offsets,
                    self.scan_tmp, self.totals, self.ranges, self.t_final, self.n_last,
                    self.emit_tmp, self.table))


def batch_items(requests, outs) -> "ctypes.Array":
    """ss_batch_item array for [(Gaussians, camera), ...] and output images."""
    arr = (_lib.SSBatchItem * len(requests))()
    for k, ((g, cam), out) in enumerate(zip(requests, outs)):
        arr[k].cam = make_camera(cam)
        arr[k].g = g.struct()
        arr[k].out_rgb = out.data_ptr()
    return arr


def batch_sizes(items, n) -> _lib.SSBatchInfo:
    info = _lib.SSBatchInfo()
    check(lib().ss_batch_sizes(items, n, ctypes.byref(info)), "ss_batch_sizes")
    return info


class BatchRenderer:
    """Renders several requests (scenes and resolutions may differ) with one
    launch per stage.  Buffers are allocated per batch through torch."""

    def __init__(self, device="cuda", growth: float = 1.25):
        self.device = torch.device(device)
        self.growth = growth

    def begin(self, requests, mode="accutile", outs=None, stream=None):
        """Stage 1 for [(Gaussians, camera), ...]; returns a handle with the
        pair count (synchronises `stream`)."""
        n = len(requests)
        if outs is None:
            outs = [torch.empty((3, int(c.height), int(c.width)), dtype=torch.float32,
                                device=self.device) for _, c in requests]
        items = batch_items(requests, outs)
        info = batch_sizes(items, n)
        frame = BatchFrame(info, n, self.device)
        fs = frame.struct()
        st = ctypes.c_void_p(stream.cuda_stream if stream is not None else
                             torch.cuda.current_stream(self.device).cuda_stream)
        counts = _lib.SSFrameCounts()
        check(lib().ss_batch_begin(items, n, mode_id(mode), ctypes.byref(fs),
                                   ctypes.byref(counts), None, st), "ss_batch_begin")
        return _BatchHandle(items, n, mode_id(mode), frame, counts, outs, st)

    def finish(self, h: "_BatchHandle"):
        """Stages 3-6; returns the output images (valid after the stream syncs)."""
        h.pairs = Pairs(int(max(h.n_pairs, 1) * self.growth) + 1024, self.device)
        fs, ps = h.frame.struct(), h.pairs.struct()
        buf = ctypes.c_int32()
        check(lib().ss_batch_finish(h.items, h.n, h.mode, ctypes.byref(fs), ctypes.byref(ps),
                                    ctypes.byref(h.counts), ctypes.byref(buf), None, h.stream),
              "ss_batch_finish")
        return h.outs

    def render(self, requests, mode="accutile", outs=None, stream=None):
        return self.finish(self.begin(requests, mode, outs, stream))


@dataclass
class _BatchHandle:
    items: object
    n: int
    mode: int
    frame: BatchFrame
    counts: _lib.SSFrameCounts
    outs: list
    stream: ctypes.c_void_p
    pairs: Pairs | None = None

    @property
    def n_pairs(self) -> int:
        return int(self.counts.n_pairs)

    @property
    def nbytes(self) -> int:
        b = self.frame.nbytes + sum(o.numel() * 4 for o in self.outs)
        if self.pairs is not None:
            b += self.pairs.capacity * 16 + self.pairs.sort_tmp.numel() * 4
        return b

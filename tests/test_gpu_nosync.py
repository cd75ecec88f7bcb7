"""ss_render_nosync (no read-back of the frame counts: the stages after the
preprocess read them on the device) against ss_render: identical sorted
pairs, ranges, images and per-pixel state; frames queued back to back; and
a pair workspace too small for the frame, which must write nothing past the
workspace, leave the background image and report the overflow."""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from gpu_util import u32

pytestmark = pytest.mark.gpu
MODES = ["3sigma", "snugbox", "accutile"]


@pytest.fixture(scope="module")
def ss():
    import paper_2412_00578_amd as ss
    ss.lib()
    return ss


def _same(a, b, p):
    assert np.array_equal(u32(a.pairs.keys[a.buf][:p]), u32(b.pairs.keys[b.buf][:p]))
    assert np.array_equal(u32(a.pairs.values[a.buf][:p]), u32(b.pairs.values[b.buf][:p]))
    assert np.array_equal(u32(a.frame.ranges), u32(b.frame.ranges))
    assert np.array_equal(a.image.cpu().numpy(), b.image.cpu().numpy())
    assert np.array_equal(a.frame.t_final.cpu().numpy(), b.frame.t_final.cpu().numpy())
    assert np.array_equal(u32(a.frame.n_last), u32(b.frame.n_last))


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("which", ["c0", "c1", "edge", "large"])
def test_nosync_equals_render(ss, gpu_device, mode, which):
    if which == "c0":
        sc, cam = scenegen.scene_c0(), scenegen.camera_c0()
    elif which == "c1":
        sc, cam = scenegen.scene_c1(), scenegen.camera_c1()
    elif which == "large":
        # Gaussians over thousands of the 14400 tiles: their emission split
        # over several waves, from the counts on the device
        sc = scenegen.scene_blobs(30_000, 31, log_s=(-3.0, 1.5))
        cam = scenegen.cameras_c1(8)[1].with_size(2560, 1440)
    else:
        sc = scenegen.scene_blobs(60_000, 21, log_s=(-3.0, 1.0))
        cam = scenegen.cameras_c1(8)[1].with_size(1920, 1080)
    print(f"[case] nosync {which} {mode}", flush=True)
    g = ss.Gaussians.from_scene(sc, gpu_device)
    ref = ss.Renderer(gpu_device).render(g, cam, mode, full=True)
    r = ss.Renderer(gpu_device)
    r.render(g, cam, mode)                 # sizes the pair workspace
    out = r.render_nosync(g, cam, mode)
    torch.cuda.synchronize()
    assert out.ok() and out.n_pairs == ref.n_pairs
    _same(out, ref, ref.n_pairs)
    if which == "c0":
        fr = oracle.render(sc, cam, mode)
        ok = ~fr.ambiguous
        assert np.abs(out.image.cpu().numpy() - fr.image)[:, ok].max() <= 1e-4


def test_frames_back_to_back(ss, gpu_device):
    """Eight frames of the benchmark scene queued with no synchronisation, then
    checked one by one against ss_render."""
    print("[case] nosync back to back", flush=True)
    sc, cams = scenegen.scene_c1(), scenegen.cameras_c1(8)
    g = ss.Gaussians.from_scene(sc, gpu_device)
    r = ss.Renderer(gpu_device)
    for c in cams:
        r.render(g, c, "accutile")
    outs = [r.render_nosync(g, c, "accutile",
                            out=torch.empty((3, c.height, c.width), device=gpu_device))
            for c in cams]
    imgs = [o.image.clone() for o in outs]
    torch.cuda.synchronize()
    ref = ss.Renderer(gpu_device)
    for c, o, im in zip(cams, outs, imgs):
        assert o.ok()
        assert np.array_equal(im.cpu().numpy(), ref.render(g, c, "accutile").cpu().numpy())


def test_workspace_overflow_is_reported(ss, gpu_device):
    print("[case] nosync overflow", flush=True)
    sc, cam = scenegen.scene_c1(), scenegen.camera_c1()
    g = ss.Gaussians.from_scene(sc, gpu_device)
    r = ss.Renderer(gpu_device)                    # no frame seen: a 1025-pair workspace
    guard = r.pairs_for(1)
    for t in guard.keys + guard.values:
        t.fill_(-7)
    out = r.render_nosync(g, cam, "accutile")
    torch.cuda.synchronize()
    assert not out.ok() and out.n_pairs > out.capacity
    assert np.all(out.image.cpu().numpy() == 0.0)                 # background only
    assert np.all(u32(out.frame.ranges) == 0)
    for t in guard.keys + guard.values:                            # nothing written
        assert np.all(t.cpu().numpy() == -7)
    r.render(g, cam, "accutile")                                   # grows the workspace
    again = r.render_nosync(g, cam, "accutile")
    torch.cuda.synchronize()
    assert again.ok()


def test_empty_scene(ss, gpu_device):
    cam = scenegen.Camera(40, 24, 40.0, 40.0, 20.0, 12.0, np.eye(3), np.zeros(3),
                          bg=(0.25, 0.5, 1.0))
    sc = scenegen.fixture_scene(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 4)),
                                np.zeros(0), np.zeros((0, 3)))
    g = ss.Gaussians.from_scene(sc, gpu_device)
    out = ss.Renderer(gpu_device).render_nosync(g, cam, "accutile")
    torch.cuda.synchronize()
    assert out.ok() and out.n_pairs == 0
    img = out.image.cpu().numpy()
    for ch, b in enumerate(cam.bg):
        assert np.all(img[ch] == np.float32(b))


def test_counts_into_pageable_memory(ss, gpu_device):
    """The frame counts land in ordinary (pageable) host memory too: the
    library falls back from the kernel's write to a copy on the stream."""
    import ctypes
    from paper_2412_00578_amd import _lib
    from paper_2412_00578_amd.render import make_camera, mode_id
    print("[case] nosync counts into pageable memory", flush=True)
    sc, cam = scenegen.scene_c0(), scenegen.camera_c0()
    g = ss.Gaussians.from_scene(sc, gpu_device)
    r = ss.Renderer(gpu_device)
    ref = r.render(g, cam, "accutile", full=True)
    c = make_camera(cam)
    frame = r.frame_for(g.n, c.width, c.height)
    pairs = r.pairs_for(max(ref.n_pairs, 1))
    out = torch.empty((3, c.height, c.width), dtype=torch.float32, device=gpu_device)
    host = np.full(2, -1, dtype=np.int64)                    # pageable
    gs, fs, ps = g.struct(), frame.struct(), pairs.struct()
    buf = ctypes.c_int32()
    st = ss.lib().ss_render_nosync(ctypes.byref(c), ctypes.byref(gs), mode_id("accutile"),
                                   ctypes.byref(fs), ctypes.byref(ps),
                                   ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(host.ctypes.data), ctypes.byref(buf), None,
                                   ctypes.c_void_p(torch.cuda.current_stream(gpu_device).cuda_stream))
    assert st == _lib.SS_OK
    torch.cuda.synchronize()
    assert host[0] == ref.n_pairs and host[1] == ref.n_visible
    assert np.array_equal(out.cpu().numpy(), ref.image.cpu().numpy())


def test_two_caller_streams(ss, gpu_device):
    """Frames queued alternately on two caller streams (two renderers, no
    synchronisation between them) share the library's colour stream: each
    frame's blend must still read its own frame's colours."""
    print("[case] nosync on two caller streams", flush=True)
    sc, cams = scenegen.scene_c1(), scenegen.cameras_c1(8)
    g = ss.Gaussians.from_scene(sc, gpu_device)
    rs = [ss.Renderer(gpu_device), ss.Renderer(gpu_device)]
    streams = [torch.cuda.Stream(device=gpu_device), torch.cuda.Stream(device=gpu_device)]
    for r in rs:
        for c in cams[:4]:
            r.render(g, c, "accutile")
    torch.cuda.synchronize()
    queued = []
    for k in range(8):
        c = cams[k % 4]
        with torch.cuda.stream(streams[k % 2]):
            out = torch.empty((3, c.height, c.width), device=gpu_device)
            queued.append((c, rs[k % 2].render_nosync(g, c, "accutile", out=out)))
    torch.cuda.synchronize()
    ref = ss.Renderer(gpu_device)
    for c, o in queued:
        assert o.ok()
        assert np.array_equal(o.image.cpu().numpy(), ref.render(g, c, "accutile").cpu().numpy())


@pytest.mark.parametrize("mode", MODES)
def test_single_call_render(ss, gpu_device, mode):
    """ss_render (one call: colour kernel on the library's second stream)
    equals the two-call render bit for bit; with a workspace smaller than the
    frame it reports the counts and SS_ERR_WORKSPACE, and work queued on the
    caller's stream afterwards still sees the frame's colours."""
    import ctypes
    from paper_2412_00578_amd import _lib
    from paper_2412_00578_amd.render import Pairs, make_camera, mode_id
    print(f"[case] single-call render {mode}", flush=True)
    sc, cam = scenegen.scene_c1(), scenegen.camera_c1()
    g = ss.Gaussians.from_scene(sc, gpu_device)
    r = ss.Renderer(gpu_device)
    ref = r.render(g, cam, mode, full=True)
    ref_img = ref.image.cpu().numpy()
    ref_rgb = ref.frame.rgb.cpu().numpy()
    c = make_camera(cam)
    frame = r.frame_for(g.n, c.width, c.height)
    stream = ctypes.c_void_p(torch.cuda.current_stream(gpu_device).cuda_stream)
    gs, fs = g.struct(), frame.struct()
    for cap in (ref.n_pairs, 1024):
        pairs = Pairs(cap, gpu_device)
        ps = pairs.struct()
        out = torch.zeros((3, c.height, c.width), device=gpu_device)
        counts = _lib.SSFrameCounts()
        buf = ctypes.c_int32(-1)
        st = ss.lib().ss_render(ctypes.byref(c), ctypes.byref(gs), mode_id(mode), ctypes.byref(fs),
                                ctypes.byref(ps), ctypes.c_void_p(out.data_ptr()),
                                ctypes.byref(counts), ctypes.byref(buf), None, stream)
        rgb = frame.rgb.clone()                      # queued on the caller's stream
        torch.cuda.synchronize()
        assert counts.n_pairs == ref.n_pairs and counts.n_visible == ref.n_visible
        vis = frame.counts.cpu().numpy() > 0
        assert np.array_equal(rgb.cpu().numpy()[vis], ref_rgb[vis])
        if cap >= ref.n_pairs:
            assert st == _lib.SS_OK
            assert np.array_equal(out.cpu().numpy(), ref_img)
        else:
            assert st == _lib.SS_ERR_WORKSPACE


def test_every_gaussian_culled(ss, gpu_device):
    """A scene whose Gaussians are all behind the camera or outside the image:
    no pairs, the background image, through the two-call, single-call and
    no-read-back renders."""
    print("[case] every Gaussian culled", flush=True)
    cam = scenegen.Camera(96, 64, 80.0, 80.0, 48.0, 32.0, np.eye(3), np.zeros(3),
                          bg=(0.1, 0.2, 0.3))
    rng = np.random.default_rng(5)
    n = 3000
    behind = np.column_stack([rng.uniform(-1, 1, n // 2), rng.uniform(-1, 1, n // 2),
                              rng.uniform(-5, -0.5, n // 2)])
    aside = np.column_stack([rng.uniform(30, 40, n - n // 2), rng.uniform(-1, 1, n - n // 2),
                             rng.uniform(2, 6, n - n // 2)])
    means = np.vstack([behind, aside])
    q = rng.normal(size=(n, 4))
    sc = scenegen.fixture_scene(means, np.full((n, 3), 0.05), q / np.linalg.norm(q, axis=1)[:, None],
                                np.full(n, 0.9), rng.uniform(0, 1, (n, 3)))
    g = ss.Gaussians.from_scene(sc, gpu_device)
    r = ss.Renderer(gpu_device)
    two = r.render(g, cam, "accutile", full=True)
    assert two.n_pairs == 0 and two.n_visible == 0
    ns = r.render_nosync(g, cam, "accutile")
    band = r.render_band(g, cam, "accutile", 1, 2)
    torch.cuda.synchronize()
    assert ns.ok() and ns.n_pairs == 0
    for img in (two.image, ns.image):
        im = img.cpu().numpy()
        for ch, b in enumerate(cam.bg):
            assert np.all(im[ch] == np.float32(b))
    bim = band.cpu().numpy()
    for ch, b in enumerate(cam.bg):
        assert np.all(bim[ch] == np.float32(b))

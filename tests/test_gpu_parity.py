"""GPU parity: every stage of the HIP pipeline against the CPU oracle.

Integers (counts, offsets, pair count, keys, values, ranges) and the FP32
records (u, v, depth, t, a, b, c) must match bit for bit; colours within
1e-6 relative; images within 1e-4 per channel except at pixels where the oracle
flags a stop decision that a different (faithful) exp could flip.
"""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from gpu_util import assert_pipeline_equal, gpu_stages, u32, u64

pytestmark = pytest.mark.gpu
MODES = ["3sigma", "snugbox", "accutile"]


@pytest.fixture(scope="module")
def ss():
    import paper_2412_00578_amd as ss
    ss.lib()
    return ss


def _run(ss, dev, scene, cam, mode):
    print(f"[case] n={scene.n} {cam.width}x{cam.height} mode={mode}", flush=True)
    r = ss.Renderer(dev, stats=True)
    g = ss.Gaussians.from_scene(scene, dev)
    return gpu_stages(r, g, cam, mode)


@pytest.mark.parametrize("mode", MODES)
def test_c0_all_stages(ss, gpu_device, mode):
    sc, cam = scenegen.scene_c0(), scenegen.camera_c0()
    gpu = _run(ss, gpu_device, sc, cam, mode)
    assert_pipeline_equal(gpu, oracle.render(sc, cam, mode))


@pytest.mark.parametrize("mode", MODES)
def test_c1_full_size(ss, gpu_device, mode):
    # 1.5M Gaussians, SH degree 3, 1600x1040: the benchmark workload.
    sc, cam = scenegen.scene_c1(), scenegen.camera_c1()
    gpu = _run(ss, gpu_device, sc, cam, mode)
    assert_pipeline_equal(gpu, oracle.render(sc, cam, mode))


@pytest.mark.parametrize("mode", ["3sigma", "accutile"])
def test_c4_largest_scene_full_hd(ss, gpu_device, mode):
    # the 6M-Gaussian resident scene of the serving workload at 1920x1080
    # (half-filled last tile row), the largest pair counts of the tests
    sc = scenegen.scene_c4(3)
    cam = scenegen.cameras_c1(8)[5].with_size(1920, 1080)
    gpu = _run(ss, gpu_device, sc, cam, mode)
    print(f"[case] pairs {gpu['n_pairs']}", flush=True)
    assert_pipeline_equal(gpu, oracle.render(sc, cam, mode))


def test_c2_shape_other_camera(ss, gpu_device):
    sc = scenegen.scene_c2()
    cam = scenegen.cameras_c2(4)[3]
    gpu = _run(ss, gpu_device, sc, cam, "accutile")
    assert_pipeline_equal(gpu, oracle.render(sc, cam, "accutile"))


@pytest.mark.parametrize("mode", MODES)
def test_partial_edge_tiles(ss, gpu_device, mode):
    # 1920x1080 has a half-filled last tile row; the camera sits inside the scene.
    sc = scenegen.scene_blobs(60_000, 21, log_s=(-3.0, 1.0))
    cam = scenegen.cameras_c1(8)[1].with_size(1920, 1080)
    gpu = _run(ss, gpu_device, sc, cam, mode)
    assert_pipeline_equal(gpu, oracle.render(sc, cam, mode))


@pytest.mark.parametrize("mode", ["3sigma", "accutile"])
def test_gaussians_over_thousands_of_tiles(ss, gpu_device, mode):
    # The camera inside a scene with scales up to e^1.5 at 2560x1440 (14400
    # tiles): hundreds of Gaussians of more than 512 tiles, whose emission is
    # split over several waves, and some covering every tile (more than
    # 16 x 512, the most runs one Gaussian is split into).  Stages only: the
    # image of 13.6M 3-sigma pairs at this size is beyond the oracle's budget
    # here, and the blend's inputs are the sorted pairs and ranges compared.
    sc = scenegen.scene_blobs(30_000, 31, log_s=(-3.0, 1.5))
    cam = scenegen.cameras_c1(8)[1].with_size(2560, 1440)
    gpu = _run(ss, gpu_device, sc, cam, mode)
    fr = oracle.render(sc, cam, mode, blend_tiles=None)
    counts = fr.records.counts.astype(np.int64)
    print(f"[case] pairs {fr.n_pairs}, over 512 tiles {(counts > 512).sum()}, "
          f"over 8192 {(counts > 8192).sum()}", flush=True)
    assert (counts > 8192).sum() > 0
    assert_pipeline_equal(gpu, fr)


def test_odd_sizes_and_sh_degrees(ss, gpu_device):
    # Ragged Gaussian count, tiny odd image, SH degree 1 and 2 stored with stride 16.
    cam = scenegen.Camera(200, 70, 180.0, 180.0, 100.0, 35.0, np.eye(3), np.zeros(3))
    for deg in (1, 2, 3):
        sc = scenegen.scene_c0(n=4097, seed=30 + deg, sh_degree=3, log_s=(-3.0, 0.8))
        sc.sh_degree = deg
        for mode in MODES:
            gpu = _run(ss, gpu_device, sc, cam, mode)
            assert_pipeline_equal(gpu, oracle.render(sc, cam, mode))


def test_sh_rows_of_odd_length(ss, gpu_device):
    # SH degree 3 stored with 17 coefficients per Gaussian: 51-float rows are
    # not 16-byte aligned, so the colour takes the LDS-staged path.
    import dataclasses
    cam = scenegen.Camera(200, 120, 180.0, 180.0, 100.0, 60.0, np.eye(3), np.zeros(3))
    sc = scenegen.scene_c0(n=5000, seed=41, sh_degree=3, log_s=(-3.0, 0.8))
    pad = np.zeros((sc.n, 1, 3), np.float32) + np.float32(0.7)   # never read (degree 3)
    sc = dataclasses.replace(sc, sh=np.ascontiguousarray(np.concatenate([sc.sh, pad], axis=1)))
    for mode in MODES:
        gpu = _run(ss, gpu_device, sc, cam, mode)
        assert_pipeline_equal(gpu, oracle.render(sc, cam, mode))


def test_degenerate_fixtures(ss, gpu_device):
    # near plane, behind the camera, non-finite, zero quaternion, sigma < 1/255,
    # a huge screen-filling Gaussian, Gaussians straddling the image edges.
    cam = scenegen.Camera(96, 80, 90.0, 90.0, 48.0, 40.0, np.eye(3), np.zeros(3))
    means = [(0, 0, 0.1), (0, 0, -3), (np.nan, 0, 3), (0, 0, 3), (0.1, 0, 3), (0, 0, 0.5),
             (-0.55, 0.2, 1.0), (0.5, -0.45, 1.0), (0.05, 0.05, 2.0), (1.9, 0, 1.0)]
    scales = [(0.05,) * 3, (0.05,) * 3, (0.05,) * 3, (0.05,) * 3, (0.05,) * 3, (2.0, 1.5, 1.0),
              (0.1, 0.02, 0.05), (0.03, 0.2, 0.05), (0.0, 0.0, 0.0), (0.5, 0.5, 0.5)]
    quats = [(1, 0, 0, 0)] * 3 + [(0, 0, 0, 0)] + [(1, 0, 0, 0)] * 2 + \
        [(0.9, 0.1, 0.2, 0.3), (0.5, -0.5, 0.5, 0.5), (1, 0, 0, 0), (1, 0, 0, 0)]
    opac = [0.5, 0.5, 0.5, 0.5, 1.0 / 300.0, 0.9, 0.8, 0.99, 0.6, 0.7]
    cols = [(0.3, 0.6, 0.9)] * 10
    sc = scenegen.fixture_scene(means, scales, quats, opac, cols)
    for mode in MODES:
        gpu = _run(ss, gpu_device, sc, cam, mode)
        assert_pipeline_equal(gpu, oracle.render(sc, cam, mode))


def test_empty_scene_gives_background(ss, gpu_device):
    cam = scenegen.Camera(40, 24, 40.0, 40.0, 20.0, 12.0, np.eye(3), np.zeros(3),
                          bg=(0.25, 0.5, 1.0))
    sc = scenegen.fixture_scene(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 4)),
                                np.zeros(0), np.zeros((0, 3)))
    r = ss.Renderer(gpu_device)
    g = ss.Gaussians.from_scene(sc, gpu_device)
    out = r.render(g, cam, "accutile", full=True)
    torch.cuda.synchronize()
    assert out.n_pairs == 0
    img = out.image.cpu().numpy()
    for ch, b in enumerate(cam.bg):
        assert np.all(img[ch] == np.float32(b))
    assert np.all(u32(out.frame.ranges) == 0)


@pytest.mark.parametrize("mode", MODES)
def test_composite_render_equals_stages(ss, gpu_device, mode):
    sc, cam = scenegen.scene_c0(seed=3), scenegen.camera_c0()
    r = ss.Renderer(gpu_device, stats=True)
    g = ss.Gaussians.from_scene(sc, gpu_device)
    stages = gpu_stages(r, g, cam, mode)
    # the composite call without per-pixel statistics renders the same bits
    out = ss.Renderer(gpu_device).render(g, cam, mode, full=True)
    torch.cuda.synchronize()
    assert out.buf == 0
    assert np.array_equal(u32(out.frame.n_last), stages["n_last"])
    p = out.n_pairs
    assert p == stages["n_pairs"]
    assert np.array_equal(u32(out.pairs.keys[0][:p]), stages["sorted_keys"])
    assert np.array_equal(u32(out.pairs.values[0][:p]), stages["sorted_values"])
    assert np.array_equal(out.image.cpu().numpy(), stages["image"])


def test_render_many_equals_frame_by_frame(ss, gpu_device):
    # pipelined frames (two frame buffers, asynchronous pair counts), with a
    # resolution change and a pair workspace that has to grow mid-sequence
    sc = scenegen.scene_c2(n=100_000)
    cams = list(scenegen.cameras_c2(5))
    cams.insert(2, cams[1].with_size(640, 480))
    cams.insert(0, cams[0].with_size(64, 48))
    g = ss.Gaussians.from_scene(sc, gpu_device)
    imgs = ss.Renderer(gpu_device).render_many(g, cams, "accutile")
    torch.cuda.synchronize()
    for k, (cam, img) in enumerate(zip(cams, imgs)):
        want = ss.Renderer(gpu_device).render(g, cam, "accutile")
        assert torch.equal(img, want), k


def test_forward_is_deterministic(ss, gpu_device):
    sc, cam = scenegen.scene_c2(n=100_000), scenegen.cameras_c2(2)[1]
    r = ss.Renderer(gpu_device)
    g = ss.Gaussians.from_scene(sc, gpu_device)
    a = r.render(g, cam, "accutile").clone()
    b = r.render(g, cam, "accutile").clone()
    assert torch.equal(a, b)


def test_snugbox_and_accutile_images_identical(ss, gpu_device):
    # The extra SnugBox pairs never pass q <= t, so the blends are bitwise equal.
    sc, cam = scenegen.scene_c1(n=300_000, seed=5), scenegen.cameras_c1(8)[2]
    r = ss.Renderer(gpu_device)
    g = ss.Gaussians.from_scene(sc, gpu_device)
    a = r.render(g, cam, "snugbox", full=True)
    ia, pa = a.image.clone(), a.n_pairs
    b = r.render(g, cam, "accutile", full=True)
    assert b.n_pairs < pa
    assert torch.equal(ia, b.image)


def test_three_modes_identical_when_t_le_9(ss, gpu_device):
    sc, cam = scenegen.scene_c0_lowsigma(), scenegen.camera_c0()
    r = ss.Renderer(gpu_device)
    g = ss.Gaussians.from_scene(sc, gpu_device)
    imgs = [r.render(g, cam, m).clone() for m in MODES]
    assert torch.equal(imgs[0], imgs[1]) and torch.equal(imgs[1], imgs[2])


# ------------------------------------------------------------ primitives alone

@pytest.mark.parametrize("n", [0, 1, 4095, 4096, 4097, 1_000_003, 6_000_000])
def test_scan_matches_cumsum(ss, gpu_device, n):
    print(f"[case] scan n={n}", flush=True)
    rng = np.random.default_rng(n + 1)
    counts = rng.integers(0, 12, size=n).astype(np.uint32)
    f = ss.Frame(n, 16, 16, gpu_device, stats=False)
    f.order_counts.copy_(torch.from_numpy(counts.view(np.int32)))
    r = ss.Renderer(gpu_device)
    total = r.scan(f, n)
    assert total == int(counts.astype(np.uint64).sum())
    if n:
        want = np.cumsum(counts, dtype=np.uint64).astype(np.uint32)
        assert np.array_equal(u32(f.offsets), want)


@pytest.mark.parametrize("n", [0, 1, 2, 255, 4095, 4097, 70_001, 1_500_000, 6_000_001])
def test_depth_order_random_keys(ss, gpu_device, n):
    print(f"[case] depth order n={n}", flush=True)
    rng = np.random.default_rng(n + 11)
    # depth bits with many exact ties, and slots without tiles (all-ones key)
    keys = rng.integers(0x3e4ccccd, 0x3e4ccccd + 20000, size=n).astype(np.uint32)
    keys[rng.random(n) < 0.2] = np.uint32(0xFFFFFFFF)
    counts = rng.integers(0, 50, size=n).astype(np.uint32)
    # tile sets: arbitrary mask and origin words, the count in word 3
    sets = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    sets[:, 3] = counts
    f = ss.Frame(n, 16, 16, gpu_device, stats=False)
    if n:
        f.depth_keys[:n].copy_(torch.from_numpy(keys.view(np.int32)))
        f.tile_sets.copy_(torch.from_numpy(sets.view(np.int32)).reshape(f.tile_sets.shape))
    r = ss.Renderer(gpu_device)
    nv = int((keys != np.uint32(0xFFFFFFFF)).sum())
    got = u32(r.depth_order(f, nv))
    torch.cuda.synchronize()
    want = np.argsort(keys, kind="stable").astype(np.uint32)[:nv]   # all-ones keys dropped
    assert np.array_equal(got, want)
    assert np.array_equal(u32(f.order_counts[:nv]), counts[want])
    # the tile sets in depth order, left at the start of the emit scratch
    assert np.array_equal(u32(f.emit_tmp[:4 * nv]).reshape(nv, 4), sets[want])


@pytest.mark.parametrize("n", [1, 63, 64, 65, 4097, 200_003])
def test_emit_random_masks(ss, gpu_device, n):
    # Every entry's tile set as an 8 x 8 mask, from single bits (0 and 63) to
    # the whole window: each entry's pair range must hold exactly its mask's
    # tiles (in any order) with its Gaussian as value.
    print(f"[case] emit masks n={n}", flush=True)
    rng = np.random.default_rng(n + 13)
    cam = scenegen.camera_c1()                      # 100 x 65 tiles
    r = ss.Renderer(gpu_device)
    # any scene of n Gaussians: the preprocess stage writes the frame's item table
    g = ss.Gaussians.from_scene(scenegen.scene_c0(n=n, seed=n % 1000), gpu_device)
    f = r.preprocess(g, cam, "accutile")
    kind = rng.integers(0, 5, size=n)
    m = (rng.integers(0, 2**32, size=n, dtype=np.uint64)
         | (rng.integers(0, 2**32, size=n, dtype=np.uint64) << np.uint64(32)))
    m = np.where(kind == 0, np.uint64(1), m)
    m = np.where(kind == 1, np.uint64(1) << np.uint64(63), m)
    m = np.where(kind == 2, np.uint64(0xFFFFFFFFFFFFFFFF), m)
    m = np.where(kind == 3, m & (m >> np.uint64(3)) & (m >> np.uint64(7)), m)
    m = np.where(m == 0, np.uint64(1) << np.uint64(5), m)
    bits = np.unpackbits(m.view(np.uint8).reshape(n, 8), axis=1, bitorder="little")
    cnt = bits.sum(1).astype(np.uint32)
    x0 = rng.integers(0, cam.tiles_x - 7, size=n).astype(np.uint32)
    y0 = rng.integers(0, cam.tiles_y - 7, size=n).astype(np.uint32)
    order = rng.permutation(n).astype(np.uint32)
    sets = np.stack([(m & np.uint64(0xFFFFFFFF)).astype(np.uint32),
                     (m >> np.uint64(32)).astype(np.uint32), x0 | (y0 << 16), cnt], 1)
    offs = np.cumsum(cnt, dtype=np.uint64).astype(np.uint32)
    n_pairs = int(offs[-1])
    f.order[:n].copy_(torch.from_numpy(order.view(np.int32)))
    f.offsets[:n].copy_(torch.from_numpy(offs.view(np.int32)))
    f.emit_tmp[:4 * n].copy_(torch.from_numpy(sets.reshape(-1).view(np.int32)))
    pairs = r.emit(cam, f, "accutile", n, n_pairs)
    torch.cuda.synchronize()
    ent, b = np.nonzero(bits)                       # entry order, bits ascending
    want_keys = (y0[ent] + b // 8) * cam.tiles_x + x0[ent] + b % 8
    seg = np.repeat(np.arange(n), cnt)
    keys = u32(pairs.keys[0][:n_pairs]).astype(np.int64)
    got = keys[np.lexsort((keys, seg))]
    want = want_keys.astype(np.int64)[np.lexsort((want_keys, seg))]
    assert np.array_equal(got, want)
    assert np.array_equal(u32(pairs.values[0][:n_pairs]), np.repeat(order, cnt))


@pytest.mark.parametrize("n", [0, 1, 2, 4095, 4097, 70_001, 5_000_003])
def test_sort_and_ranges_random_keys(ss, gpu_device, n):
    print(f"[case] sort n={n}", flush=True)
    rng = np.random.default_rng(n + 7)
    cam = scenegen.Camera(1600, 1040, 1000.0, 1000.0, 800.0, 520.0, np.eye(3), np.zeros(3))
    n_tiles = cam.tiles_x * cam.tiles_y
    keys = rng.integers(0, n_tiles, size=n).astype(np.uint32)
    vals = rng.permutation(n).astype(np.uint32)    # arbitrary values: checks stability
    r = ss.Renderer(gpu_device)
    pairs = r.pairs_for(n)
    if n:
        pairs.keys[0][:n].copy_(torch.from_numpy(keys.view(np.int32)))
        pairs.values[0][:n].copy_(torch.from_numpy(vals.view(np.int32)))
    ob = r.sort(cam, pairs, n, 0)
    f = ss.Frame(1, cam.width, cam.height, gpu_device, stats=False)
    r.ranges(cam, f, pairs, n, ob)
    torch.cuda.synchronize()
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(u32(pairs.keys[ob][:n]), keys[order])
    assert np.array_equal(u32(pairs.values[ob][:n]), vals[order])
    st = keys[order].astype(np.int64)
    rg = u32(f.ranges).reshape(-1, 2)
    assert np.array_equal(rg[:, 0], np.searchsorted(st, np.arange(n_tiles), "left"))
    assert np.array_equal(rg[:, 1], np.searchsorted(st, np.arange(n_tiles), "right"))

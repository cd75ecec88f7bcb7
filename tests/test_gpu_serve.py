"""Batched rendering and the serving loop on the GPU.

Every image rendered inside a batch (scenes and resolutions mixed) or served
from a request stream must be bit-identical to rendering the request alone,
and a batched item must match the oracle like a single frame does."""
import numpy as np
import pytest
import torch

import oracle
import scenegen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ss():
    import paper_2412_00578_amd as ss
    ss.lib()
    return ss


@pytest.fixture(scope="module")
def scenes(ss, gpu_device):
    specs = [(20_000, 50), (60_000, 51), (150_000, 52)]
    host = [scenegen.scene_blobs(n, seed, log_s=(-3.5, 1.0)) for n, seed in specs]
    return host, [ss.Gaussians.from_scene(s, gpu_device) for s in host]


def _cams(seed, k):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(k):
        w, h = scenegen.C4_RESOLUTIONS[int(rng.integers(0, 4))]
        out.append(scenegen.random_orbit_cameras(rng, 1, 12.0, w, h)[0])
    return out


def _alone(ss, dev, g, cam, mode):
    return ss.Renderer(dev).render(g, cam, mode).clone()


@pytest.mark.parametrize("mode", ["3sigma", "accutile"])
def test_batch_equals_alone(ss, gpu_device, scenes, mode):
    _, gs = scenes
    cams = _cams(7, 6)
    reqs = [(gs[k % 3], cams[k]) for k in range(6)] + [(gs[0], cams[0])]
    print(f"[case] batch of {len(reqs)} mode={mode}", flush=True)
    outs = ss.BatchRenderer(gpu_device).render(reqs, mode)
    torch.cuda.synchronize()
    for (g, cam), img in zip(reqs, outs):
        assert torch.equal(img, _alone(ss, gpu_device, g, cam, mode))


def test_batch_item_matches_oracle(ss, gpu_device, scenes):
    host, gs = scenes
    cams = _cams(11, 3)
    reqs = [(gs[2], cams[0]), (gs[0], cams[1]), (gs[1], cams[2])]
    outs = ss.BatchRenderer(gpu_device).render(reqs, "accutile")
    torch.cuda.synchronize()
    for (k, cam), img in zip([(2, cams[0]), (0, cams[1]), (1, cams[2])], outs):
        fr = oracle.render(host[k], cam, "accutile")
        ok = ~fr.ambiguous
        assert np.abs(img.cpu().numpy() - fr.image)[:, ok].max() <= 1e-4


@pytest.mark.parametrize("mode", ["3sigma", "accutile"])
def test_batch_with_gaussians_over_thousands_of_tiles(ss, gpu_device, scenes, mode):
    # A camera inside a scene of large Gaussians at 2560x1440 (some cover all
    # 14400 tiles, so their emission is split over several waves) batched with
    # the same scene at 1600x1040 and another scene: every image bit-identical
    # to the request rendered alone.
    _, gs = scenes
    big = ss.Gaussians.from_scene(scenegen.scene_blobs(30_000, 31, log_s=(-3.0, 1.5)),
                                  gpu_device)
    cam = scenegen.cameras_c1(8)[1]
    reqs = [(gs[2], _cams(17, 1)[0]), (big, cam.with_size(2560, 1440)), (big, cam)]
    print(f"[case] batch with large Gaussians mode={mode}", flush=True)
    outs = ss.BatchRenderer(gpu_device).render(reqs, mode)
    torch.cuda.synchronize()
    for (g, c), img in zip(reqs, outs):
        assert torch.equal(img, _alone(ss, gpu_device, g, c, mode))


def test_batch_with_empty_and_tiny_scenes(ss, gpu_device, scenes):
    _, gs = scenes
    empty = scenegen.fixture_scene(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 4)),
                                   np.zeros(0), np.zeros((0, 3)))
    one = scenegen.fixture_scene([(0.0, 0.0, 3.0)], [(0.2, 0.1, 0.1)], [(1, 0, 0, 0)], [0.8],
                                 [(1.0, 0.5, 0.2)])
    ge, go = ss.Gaussians.from_scene(empty, gpu_device), ss.Gaussians.from_scene(one, gpu_device)
    cam = scenegen.Camera(100, 60, 80.0, 80.0, 50.0, 30.0, np.eye(3), np.zeros(3))
    cams = _cams(13, 2)
    reqs = [(ge, cam), (gs[1], cams[0]), (go, cam), (ge, cams[1]), (go, cams[1])]
    outs = ss.BatchRenderer(gpu_device).render(reqs, "accutile")
    torch.cuda.synchronize()
    for (g, c), img in zip(reqs, outs):
        assert torch.equal(img, _alone(ss, gpu_device, g, c, "accutile"))


def test_served_stream_equals_alone(ss, gpu_device, scenes):
    from paper_2412_00578_amd.serve import Request, serve
    _, gs = scenes
    stream = scenegen.request_stream(40, qps=2000.0, n_scenes=3, seed=5)
    reqs = [Request(k, s, cam, t) for k, (t, s, cam) in enumerate(stream)]
    st = serve(gs, reqs, gpu_device, "accutile", pool_bytes=2 << 30, max_batch=6,
               keep_images=True)
    torch.cuda.synchronize()
    print(f"[serve] {st.summary()}", flush=True)
    assert st.failed == 0 and all(r.status == "done" for r in reqs)
    assert max(st.batch_sizes) > 1
    for r in reqs:
        assert torch.equal(r.image, _alone(ss, gpu_device, gs[r.scene], r.cam, "accutile")), r.rid
    assert np.isfinite(st.pct(99)) and st.pct(50) > 0

"""The tile-band viewport: one band of tile rows of a frame, rendered on its
own (the piece of a frame one GPU renders when a frame is split across GPUs
by screen-space bands), against the oracle's whole frame restricted to the
band and against the GPU's own whole-frame render.

Pairs (tile ids relative to the band), values, per-tile ranges and per-
Gaussian band counts are bit-exact against the oracle; the band's image rows
are bit-identical to the same rows of the whole-frame render and within
1e-4 of the oracle's where the oracle fixes the decisions."""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from gpu_util import MIN_COMPARED, u32

pytestmark = pytest.mark.gpu
MODES = ["3sigma", "snugbox", "accutile"]


@pytest.fixture(scope="module")
def ss():
    import paper_2412_00578_amd as ss
    ss.lib()
    return ss


def band_expectation(fr, cam, row0, rows):
    """The oracle frame restricted to tile rows [row0, row0 + rows)."""
    tiles = (fr.sorted_keys >> np.uint64(32)).astype(np.int64)
    ty = tiles // cam.tiles_x
    keep = (ty >= row0) & (ty < row0 + rows)
    keys = (tiles[keep] - row0 * cam.tiles_x).astype(np.uint32)
    vals = fr.sorted_values[keep]
    t0, t1 = row0 * cam.tiles_x, (row0 + rows) * cam.tiles_x
    first = int(np.searchsorted(tiles, t0, "left"))
    ranges = (fr.ranges[t0:t1].astype(np.int64) - first).astype(np.uint32)
    counts = np.bincount(vals, minlength=fr.records.n).astype(np.uint32)
    return keys, vals, ranges, counts


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("size,band", [((1600, 1040), (30, 8)), ((1600, 1040), (0, 9)),
                                       ((1920, 1080), (61, 7)), ((1920, 1080), (67, 1))])
def test_band_matches_whole_frame(ss, gpu_device, mode, size, band):
    row0, rows = band
    sc = scenegen.scene_blobs(60_000, 21, log_s=(-3.0, 1.0))
    cam = scenegen.cameras_c1(8)[1].with_size(*size)
    print(f"[case] band rows [{row0}, {row0 + rows}) of {size} mode={mode}", flush=True)
    g = ss.Gaussians.from_scene(sc, gpu_device)
    r = ss.Renderer(gpu_device)
    out = r.render_band(g, cam, mode, row0, rows, full=True)
    whole = ss.Renderer(gpu_device).render(g, cam, mode)
    torch.cuda.synchronize()
    fr = oracle.render(sc, cam, mode)
    keys, vals, ranges, counts = band_expectation(fr, cam, row0, rows)
    p = out.n_pairs
    assert p == len(keys)
    assert np.array_equal(u32(out.frame.counts), counts)
    assert np.array_equal(u32(out.pairs.keys[out.buf][:p]), keys)
    assert np.array_equal(u32(out.pairs.values[out.buf][:p]), vals)
    assert np.array_equal(u32(out.frame.ranges).reshape(-1, 2), ranges)
    y0, y1 = 16 * row0, min(cam.height, 16 * (row0 + rows))
    img = out.image.cpu().numpy()
    assert img.shape == (3, y1 - y0, cam.width)
    assert np.array_equal(img, whole[:, y0:y1].cpu().numpy())
    ok = ~fr.ambiguous[y0:y1]
    d = np.abs(img - fr.image[:, y0:y1])[:, ok]
    assert d.max(initial=0.0) <= 1e-4, d.max()
    assert ok.mean() >= MIN_COMPARED


@pytest.mark.parametrize("mode", ["3sigma", "accutile"])
def test_band_of_large_gaussians(ss, gpu_device, mode):
    # A band of a 2560x1440 view from inside a scene of large Gaussians (some
    # cover every tile, so their emission in the band is split over several
    # waves): pairs, counts and ranges as the oracle's frame restricted to the
    # band, image rows bit-identical to the whole frame's (the oracle's image
    # of this frame is beyond its budget here).
    row0, rows = 40, 30
    sc = scenegen.scene_blobs(30_000, 31, log_s=(-3.0, 1.5))
    cam = scenegen.cameras_c1(8)[1].with_size(2560, 1440)
    print(f"[case] band rows [{row0}, {row0 + rows}) of large Gaussians mode={mode}", flush=True)
    g = ss.Gaussians.from_scene(sc, gpu_device)
    out = ss.Renderer(gpu_device).render_band(g, cam, mode, row0, rows, full=True)
    whole = ss.Renderer(gpu_device).render(g, cam, mode)
    torch.cuda.synchronize()
    fr = oracle.render(sc, cam, mode, blend_tiles=None)
    keys, vals, ranges, counts = band_expectation(fr, cam, row0, rows)
    p = out.n_pairs
    assert p == len(keys)
    assert np.array_equal(u32(out.frame.counts), counts)
    assert np.array_equal(u32(out.pairs.keys[out.buf][:p]), keys)
    assert np.array_equal(u32(out.pairs.values[out.buf][:p]), vals)
    assert np.array_equal(u32(out.frame.ranges).reshape(-1, 2), ranges)
    img = out.image.cpu().numpy()
    assert np.array_equal(img, whole[:, 16 * row0:16 * (row0 + rows)].cpu().numpy())


def test_bands_tile_the_frame(ss, gpu_device):
    """Eight bands of the 1.5M-Gaussian benchmark frame (AccuTile) together
    hold exactly the whole frame's pairs, and their images stack into the
    whole image bit for bit."""
    sc, cam = scenegen.scene_c1(), scenegen.camera_c1()
    print("[case] 8 bands of the benchmark frame", flush=True)
    g = ss.Gaussians.from_scene(sc, gpu_device)
    whole = ss.Renderer(gpu_device).render(g, cam, "accutile", full=True)
    torch.cuda.synchronize()
    wk = u32(whole.pairs.keys[whole.buf][:whole.n_pairs])
    wv = u32(whole.pairs.values[whole.buf][:whole.n_pairs])
    r = ss.Renderer(gpu_device)
    bounds = np.linspace(0, cam.tiles_y, 9).round().astype(int)
    imgs, total = [], 0
    for b0, b1 in zip(bounds[:-1], bounds[1:]):
        out = r.render_band(g, cam, "accutile", int(b0), int(b1 - b0), full=True)
        torch.cuda.synchronize()
        p = out.n_pairs
        sel = (wk // cam.tiles_x >= b0) & (wk // cam.tiles_x < b1)
        assert np.array_equal(u32(out.pairs.keys[out.buf][:p]), wk[sel] - b0 * cam.tiles_x)
        assert np.array_equal(u32(out.pairs.values[out.buf][:p]), wv[sel])
        imgs.append(out.image.cpu().numpy())
        total += p
    assert total == whole.n_pairs
    assert np.array_equal(np.concatenate(imgs, axis=1), whole.image.cpu().numpy())

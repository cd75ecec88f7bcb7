"""Helpers shared by the GPU tests: run the HIP pipeline stage by stage and
compare every intermediate with the oracle."""
import numpy as np
import torch

import oracle


def u32(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def u64(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


def gpu_stages(renderer, g, cam, mode):
    """Runs the stages one call at a time; returns every intermediate."""
    frame = renderer.preprocess(g, cam, mode)
    torch.cuda.synchronize()
    out = {
        "geom": frame.geom.cpu().numpy().copy(),
        "conic": frame.conic.cpu().numpy().copy(),
        "rgb": frame.rgb.cpu().numpy().copy(),
        "counts": u32(frame.counts).copy(),
        "tile_sets": u32(frame.tile_sets).copy(),
        "tiles_x": int(cam.tiles_x),
        "tiles_y": int(cam.tiles_y),
        "mode": mode,
    }
    out["depth_keys"] = u32(frame.depth_keys[:frame.n]).copy()
    p_pre, nv = renderer.counts(frame)
    out["n_visible"] = nv
    out["n_pairs_pre"] = p_pre
    out["order"] = u32(renderer.depth_order(frame, nv)).copy()
    torch.cuda.synchronize()
    out["order_counts"] = u32(frame.order_counts[:nv]).copy()
    p = renderer.scan(frame, nv)
    out["n_pairs"] = p
    out["offsets"] = u32(frame.offsets[:nv]).copy()
    pairs = renderer.emit(cam, frame, mode, nv, p, buf=0)
    torch.cuda.synchronize()
    out["keys"] = u32(pairs.keys[0][:p]).copy()
    out["values"] = u32(pairs.values[0][:p]).copy()
    ob = renderer.sort(cam, pairs, p, 0)
    renderer.ranges(cam, frame, pairs, p, ob)
    img = renderer.blend(cam, frame, pairs, ob)
    torch.cuda.synchronize()
    out["sorted_keys"] = u32(pairs.keys[ob][:p]).copy()
    out["sorted_values"] = u32(pairs.values[ob][:p]).copy()
    out["ranges"] = u32(frame.ranges).copy()
    out["image"] = img.cpu().numpy()
    out["t_final"] = frame.t_final.cpu().numpy().copy()
    out["n_last"] = u32(frame.n_last).copy()
    out["n_eval"] = u32(frame.n_eval).copy()
    out["n_contrib"] = u32(frame.n_contrib).copy()
    return out


def first_diffs(a, b, k=5):
    idx = np.nonzero(a != b)[0][:k]
    return [(int(i), a[i], b[i]) for i in idx]


def assert_records_equal(gpu, ref: "oracle.Records"):
    g32, r32 = gpu["geom"].view(np.uint32), ref.geom.view(np.uint32)
    bad = np.nonzero((g32 != r32).any(axis=1))[0]
    assert len(bad) == 0, f"{len(bad)} geom mismatches, e.g. " + str(
        [(int(i), gpu["geom"][i].tolist(), ref.geom[i].tolist()) for i in bad[:3]])
    c32, q32 = gpu["conic"].view(np.uint32), ref.conic.view(np.uint32)
    bad = np.nonzero((c32 != q32).any(axis=1))[0]
    assert len(bad) == 0, f"{len(bad)} conic mismatches, e.g. " + str(
        [(int(i), gpu["conic"][i].tolist(), ref.conic[i].tolist()) for i in bad[:3]])
    # colours are compared where the record has tiles: the GPU evaluates the
    # view-dependent colour only for Gaussians that can be blended
    has = ref.counts > 0
    np.testing.assert_allclose(gpu["rgb"][has], ref.rgb[has], rtol=1e-6, atol=2e-6)
    bad = np.nonzero(gpu["counts"] != ref.counts)[0]
    assert len(bad) == 0, f"{len(bad)} count mismatches " + str(first_diffs(gpu["counts"],
                                                                            ref.counts))


CULLED_KEY = np.uint32(0xFFFFFFFF)

# Floor on the fraction of pixels the image comparison covers: the oracle
# excludes only pixels whose inclusion or stop decision lies inside an FP32
# rounding band (at most 0.1 % of any tested frame).
MIN_COMPARED = 0.999


def expected_depth_keys(rec: "oracle.Records") -> np.ndarray:
    """Depth-order key of every record: bits(depth), or all ones without tiles."""
    bits = np.ascontiguousarray(rec.geom[:, 2]).view(np.uint32)
    return np.where(rec.counts > 0, bits, CULLED_KEY).astype(np.uint32)


def expected_order(dkeys: np.ndarray) -> np.ndarray:
    """Indices sorted by (key, index)."""
    return np.lexsort((np.arange(len(dkeys)), dkeys)).astype(np.uint32)


def segment_sorted(keys, counts_in_order):
    """Keys with each Gaussian's run (lengths counts_in_order) sorted: the order
    of a Gaussian's own pairs is unspecified."""
    c = counts_in_order.astype(np.int64)
    seg = np.repeat(np.arange(len(c)), c)
    return keys[np.lexsort((keys, seg))]


def assert_tile_sets(tsets, fr, tiles_x, tiles_y, mode):
    """Every stored tile mask expands to exactly the oracle's tile list, and a
    Gaussian with tiles but without a mask has a tile rectangle wider or taller
    than 8 tiles (the rectangle, not the tile list: an AccuTile list can miss a
    corner tile of its rectangle)."""
    counts = fr.records.counts.astype(np.int64)
    mask = tsets[:, 0].astype(np.uint64) | (tsets[:, 1].astype(np.uint64) << np.uint64(32))
    x0, y0 = (tsets[:, 2] & 0xFFFF).astype(np.int64), (tsets[:, 2] >> 16).astype(np.int64)
    has = mask != 0
    assert not np.any(has & (counts == 0))
    # oracle tiles, each Gaussian's run ascending
    tiles = segment_sorted((fr.keys >> np.uint64(32)).astype(np.int64), counts)
    owner = np.repeat(np.arange(len(counts)), counts)
    # masked Gaussians: bits in ascending order give ascending tile ids
    g, b = np.nonzero(((mask[has, None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)) != 0)
    gi = np.nonzero(has)[0][g]
    got = (y0[gi] + b // 8) * tiles_x + x0[gi] + b % 8
    assert np.array_equal(got, tiles[has[owner]])
    # unmasked Gaussians with tiles: their tile rectangle exceeds 8 on a side
    rec = fr.records
    for i in np.nonzero((~has) & (counts > 0))[0]:
        x0r, y0r, x1r, y1r = oracle.tile_rect(rec.geom[i], rec.conic[i], mode, tiles_x, tiles_y)
        assert x1r - x0r >= 8 or y1r - y0r >= 8, (int(i), (x0r, y0r, x1r, y1r))


def depth_ordered_pairs(fr, order):
    """The oracle's pairs (emitted in index order, each Gaussian's tiles in its
    enumeration order) regrouped Gaussian by Gaussian in `order`: the pairs the
    depth-ordered emission writes, with key = tile id."""
    counts = fr.records.counts.astype(np.int64)
    start = np.cumsum(counts) - counts
    c = counts[order]
    seg0 = np.repeat(start[order], c)
    within = np.arange(int(c.sum())) - np.repeat(np.cumsum(c) - c, c)
    idx = seg0 + within
    return (fr.keys[idx] >> np.uint64(32)).astype(np.uint32), fr.values[idx].astype(np.uint32)


def assert_pipeline_equal(gpu, fr, image_tol=1e-4):
    """Bit-exact integer intermediates; image within image_tol except where the
    oracle flags a stop decision that exp rounding may flip.

    The oracle sorts (tile << 32 | depth, index) pairs once; the GPU path orders
    the Gaussians by depth first, emits tile-id keys in that order and sorts
    them stably by tile.  The expected GPU intermediates are derived from the
    oracle's: the final sorted values and ranges must be identical."""
    assert_records_equal(gpu, fr.records)
    assert_tile_sets(gpu["tile_sets"], fr, gpu["tiles_x"], gpu["tiles_y"], gpu["mode"])
    dk = expected_depth_keys(fr.records)
    assert np.array_equal(gpu["depth_keys"], dk), first_diffs(gpu["depth_keys"], dk)
    nv = int((fr.records.counts > 0).sum())
    assert gpu["n_visible"] == nv
    assert gpu["n_pairs_pre"] == fr.n_pairs
    order = expected_order(dk)[:nv]         # Gaussians without tiles sort last
    assert np.array_equal(gpu["order"], order), first_diffs(gpu["order"], order)
    assert np.array_equal(gpu["order_counts"], fr.records.counts[order])
    assert gpu["n_pairs"] == fr.n_pairs
    counts = fr.records.counts.astype(np.uint64)
    assert np.array_equal(gpu["offsets"], np.cumsum(counts[order]).astype(np.uint32))
    cio = counts[order]
    ek, ev = depth_ordered_pairs(fr, order)
    gk, ek = segment_sorted(gpu["keys"], cio), segment_sorted(ek, cio)
    assert np.array_equal(gk, ek), first_diffs(gk, ek)
    assert np.array_equal(gpu["values"], ev), first_diffs(gpu["values"], ev)
    st = (fr.sorted_keys >> np.uint64(32)).astype(np.uint32)
    assert np.array_equal(gpu["sorted_keys"], st), first_diffs(gpu["sorted_keys"], st)
    assert np.array_equal(gpu["sorted_values"], fr.sorted_values)
    assert np.array_equal(gpu["ranges"], fr.ranges)
    if fr.image is not None:
        ok = ~fr.ambiguous
        d = np.abs(gpu["image"] - fr.image)[:, ok]
        assert d.max(initial=0.0) <= image_tol, f"image max diff {d.max()}"
        assert np.abs(gpu["t_final"] - fr.t_final)[ok].max(initial=0.0) <= 1e-5
        assert np.array_equal(gpu["n_last"][ok], fr.n_last[ok])
        assert np.array_equal(gpu["n_eval"][ok], fr.n_eval[ok])
        assert np.array_equal(gpu["n_contrib"][ok], fr.n_contrib[ok])
        print(f"[parity] compared pixels {ok.mean():.6f} "
              f"({int((~ok).sum())} flagged ambiguous of {ok.size})", flush=True)
        assert ok.mean() >= MIN_COMPARED

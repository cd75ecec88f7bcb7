#!/usr/bin/env python3
"""Forward-render benchmark on one MI355X.

Workload: a 1.5M-Gaussian SH-degree-3 clustered scene (200 anisotropic blobs
plus 10% uniform background in a 20-unit box) rendered at 1600x1040 with 16x16
tiles from 8 orbit cameras (radius 12, 10 degrees elevation), all synthetic and
seeded.  One step is one forward render of one frame: preprocess, depth
order, scan, key emission, tile sort, tile ranges and blend, timed frame after
frame (the paper's per-frame timing); the stages after the preprocess read
the frame counts on the device (ss_render_nosync), and the same frames with
the counts read back to the host mid-frame (ss_render) are reported beside.  `value` is the AccuTile frame rate measured
that way; each of the three tile assignments (3-sigma, SnugBox, AccuTile) is
timed over the same frames of the same scene, and their ratios stand beside
the paper's (Table 2: 1.82x SnugBox, 1.99x AccuTile on an RTX A5000).  The
same frames rendered as one pipelined sequence (consecutive frames' stages
overlapping on three streams, the host never waiting) are reported as a
throughput beside it.

Per-stage kernel times come from hipEvents the library records on its stream
inside every timed frame.  The blend (the dominant kernel) is reported against
the FP32 VALU roofline, the other stages against 8 TB/s of HBM, and the frame
as the sum of the stages' roofline times over the measured frame time.  Also
measured: the 150k-Gaussian scene over 64 orbit cameras (cost per
Gaussian-tile pair and per evaluated pixel-Gaussian pair), the
differentiable 1M-Gaussian 1264x832 forward + backward with an L1 loss, the
adjoint kernels against their rooflines, a serving run, and the CPU oracle on
one core and on all the host's cores.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline] [--no-serve]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "render FPS (AccuTile vs 3-sigma) at 1.5M Gaussians 1600px; p50/p99 serve ms"
MODES = ("3sigma", "snugbox", "accutile")

# Roofline constants (MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz; packed
# FP32 is not used, so one FP32 VALU op per lane per clock).
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12      # 39.3 T ops/s
PEAK_HBM_GBS = 8000.0
# Blend work.  Per evaluated (pixel, Gaussian) pair the method computes dx, dy,
# the quadratic form (a dx dx, (2b) dx, two fused multiply-adds) and the q <= t
# test; per blended pair the exponent scale, exp, sigma * exp, the 0.99 clamp,
# 1 - alpha, T (1 - alpha), alpha T, the stop test and three colour FMAs.  The
# exp issues at a quarter of the rate (4 issue slots).
#   RATED_SLOTS_PER_EVAL: the unit the measurement plan rates the blend in,
#     about 17 VALU lane-ops + one exp per evaluated pair (21 slots), charged
#     to every evaluated pair;
#   SLOTS_PER_EVAL / SLOTS_PER_BLENDED: the count above, with the exp and the
#     blending work charged only to pairs that pass the test.
RATED_SLOTS_PER_EVAL = 21
SLOTS_PER_EVAL, SLOTS_PER_BLENDED = 8, 13
# The blend adjoint walks each pixel's list back from its last blended entry;
# it is rated at about twice the forward's slots per walked entry.
RATED_SLOTS_PER_WALKED = 42
# Algorithmic HBM bytes: the geometry kernel reads 44 B (mean, scale,
# quaternion, opacity) and writes 56 B (geom, conic, count, depth key, tile
# set) per Gaussian, the colour kernel reads the count and writes rgb (20 B) per
# Gaussian and reads the mean and the SH-3 row (204 B) of each Gaussian with
# tiles; the depth order moves 8 B per slot in its compacting first pass plus
# 100 B per Gaussian with tiles over all four passes (keys, values, and the
# last pass's gather of the tile sets into depth order); the scan reads the
# counts twice and writes the offsets (12 B per Gaussian with tiles); the emit
# stage reads 28 B per Gaussian with tiles and writes 8 B per pair; the tile
# sort moves 20 B per pair per pass; the ranges read 4 B per pair and write
# 8 B per tile; the blend gathers a 44-B record per pair and writes 20 B per
# pixel.
PRE_BYTES_PER_G = 44 + 56
COLOUR_BYTES_PER_G, COLOUR_BYTES_PER_VISIBLE = 20, 204
DEPTH_ORDER_BYTES_PER_SLOT, DEPTH_ORDER_BYTES_PER_VISIBLE = 8, 100
SCAN_BYTES_PER_VISIBLE = 12
EMIT_BYTES_PER_VISIBLE, EMIT_BYTES_PER_PAIR = 28, 8
SORT_BYTES_PER_PAIR_PASS = 20
RANGES_BYTES_PER_PAIR, RANGES_BYTES_PER_TILE = 4, 8
# The preprocess adjoint reads the parameters (44 B), the record (32 B) and
# the screen-space gradients (48 B) of every Gaussian and the SH-3 row (192 B)
# of each Gaussian with tiles, and writes 59 floats of gradients per Gaussian.
PBWD_BYTES_PER_G, PBWD_BYTES_PER_VISIBLE = 44 + 32 + 48 + 236, 192
PAPER = {"hardware": "NVIDIA RTX A5000", "source": "Table 2 (FPS = 1000 / Table 1 overall ms)",
         "fps": {"3sigma": 134, "snugbox": 244, "accutile": 267},
         "speedup_vs_3sigma": {"snugbox": 1.82, "accutile": 1.99}}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def blend_traffic():
    """HBM bytes (read + written) per launch of the blend (k_blend<false>,
    AccuTile frame) from the committed FETCH_SIZE / WRITE_SIZE counter summary,
    calibrated against a plain copy; None when that summary was taken on
    another version of the blend source (its sha256 differs) or is missing."""
    root = os.path.dirname(os.path.abspath(__file__))
    src = os.path.join(root, "paper_2412_00578_amd", "csrc", "k_blend.hip")
    summary = os.path.join(root, "profiles", "forward_c1_hbm_traffic.txt")
    try:
        text = open(summary).read().splitlines()
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    if not any(line.strip() == f"k_blend source sha256: {digest}" for line in text):
        return None
    for line in text:
        f = line.split()
        if f and f[0] == "k_blend<false>" and len(f) >= 4:
            return int(round((float(f[2]) + float(f[3])) * 2**20))
    return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(scene, cam, runs=3):
    """The oracle (plain C, one thread) rendering one AccuTile frame."""
    import oracle
    oracle.lib()
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        oracle.render(scene, cam, "accutile")
        times.append(time.perf_counter() - t0)
        log(f"  cpu oracle frame, 1 core: {times[-1]:.2f} s")
    ms = statistics.median(times) * 1e3
    return {"value": round(1000.0 / ms, 4), "unit": "FPS", "cores": 1, "kind": "oracle",
            "sample": f"one full 1600x1040 AccuTile frame of the 1.5M-Gaussian scene "
                      f"(camera 0), median of {runs} runs, {ms:.0f} ms/frame, one thread, "
                      f"on {cpu_model()} ({host_cores()} cores available)"}


# Worker state of the all-cores oracle run, set before the pools fork.
_POOL = {}


def _pool_preprocess(span):
    import dataclasses
    import oracle
    lo, hi = span
    sc = _POOL["scene"]
    sub = dataclasses.replace(sc, means=sc.means[lo:hi], scales=sc.scales[lo:hi],
                              quats=sc.quats[lo:hi], opacity=sc.opacity[lo:hi], sh=sc.sh[lo:hi])
    rec = oracle.preprocess(sub, _POOL["cam"], _POOL["mode"])
    return rec.geom, rec.conic, rec.rgb, rec.counts, rec.visible


def _pool_blend(rows):
    import oracle
    cam = _POOL["cam"]
    tiles = [ty * cam.tiles_x + tx for ty in range(rows[0], rows[1]) for tx in range(cam.tiles_x)]
    img = oracle.blend(cam, _POOL["ranges"], _POOL["values"], _POOL["rec"], tiles)[0]
    y0, y1 = rows[0] * 16, min(cam.height, rows[1] * 16)
    return y0, img[:, y0:y1].copy()


def oracle_frame_all_cores(scene, cam, mode, cores):
    """One oracle frame with its per-Gaussian and per-tile stages spread over a
    process pool: the preprocess over chunks of Gaussians and the blend over
    tile rows; emission, the pair sort and the ranges run in the parent."""
    import multiprocessing as mp

    import numpy as np
    import oracle
    ctx = mp.get_context("fork")
    _POOL.clear()
    _POOL.update(scene=scene, cam=cam, mode=mode)
    n = scene.n
    cuts = np.linspace(0, n, 4 * cores + 1).astype(np.int64)
    with ctx.Pool(cores) as pool:
        parts = pool.map(_pool_preprocess, list(zip(cuts[:-1], cuts[1:])))
    rec = oracle.Records(np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts]),
                         np.concatenate([p[2] for p in parts]), np.concatenate([p[3] for p in parts]),
                         oracle.mode_id(mode), sum(p[4] for p in parts))
    keys, vals = oracle.emit(rec, cam)
    skeys, svals = oracle.sort_pairs(keys, vals)
    ranges = oracle.tile_ranges(skeys, cam.tiles_x * cam.tiles_y)
    _POOL.update(rec=rec, ranges=ranges, values=svals)
    img = np.zeros((3, cam.height, cam.width), np.float32)
    rows = [(r, min(r + 1, cam.tiles_y)) for r in range(cam.tiles_y)]
    with ctx.Pool(cores) as pool:
        for y0, part in pool.imap_unordered(_pool_blend, rows):
            img[:, y0:y0 + part.shape[1]] = part
    _POOL.clear()
    return img, len(skeys)


def cpu_baseline_all_cores(scene, cam, runs=3):
    cores = host_cores()
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        oracle_frame_all_cores(scene, cam, "accutile", cores)
        times.append(time.perf_counter() - t0)
        log(f"  cpu oracle frame, {cores} processes: {times[-1]:.2f} s")
    ms = statistics.median(times) * 1e3
    return {"value": round(1000.0 / ms, 4), "unit": "FPS", "cores": cores, "kind": "oracle",
            "sample": f"the same frame with the oracle's preprocess (chunks of Gaussians) and "
                      f"blend (tile rows) spread over {cores} processes, emission, pair sort "
                      f"and ranges in one; median of {runs} runs, {ms:.0f} ms/frame, on "
                      f"{cpu_model()}"}


def work_counters(ss, g, cams, mode):
    """Pairs, Gaussians with tiles, evaluated and blended pixel-Gaussian pairs
    per camera (statistics variant of the blend, untimed)."""
    import torch
    r = ss.Renderer(g.device, stats=True)
    P, V, E, I = [], [], [], []
    for cam in cams:
        out = r.render(g, cam, mode, full=True)
        torch.cuda.synchronize()
        P.append(out.n_pairs)
        V.append(out.n_visible)
        E.append(int(out.frame.n_eval.to(torch.int64).sum().item()))
        I.append(int(out.frame.n_contrib.to(torch.int64).sum().item()))
    return P, V, E, I


def time_frames(ss, r, g, cams, mode, steps, warmup, band=None, sync=False):
    """Frames one by one, each a complete forward render of one camera.  The
    frame time is measured over `steps` frames rendered back to back and
    bracketed by two events (no events inside a frame); the stage times come
    from a second pass over the same frames in which the library records its
    nine stage events inside every frame (each recorded event costs the
    stream a few microseconds).  Whole frames use ss_render_nosync (the host
    queues each frame whole; every frame is checked afterwards to have fit
    its pair workspace), or with sync=True ss_render, which reads the frame
    counts back mid-frame.  Returns (mean ms per frame, mean stage ms, mean ms
    per frame of the second pass)."""
    import torch
    dev = g.device
    c0 = cams[0]
    outs = [torch.empty((3, c0.height, c0.width), dtype=torch.float32, device=dev)
            for _ in range(2)]
    queued = []

    def frame(k, events=None):
        cam = cams[k % len(cams)]
        if band is not None:
            r.render_band(g, cam, mode, band[0], band[1], events=events)
        elif sync:
            r.render(g, cam, mode, out=outs[k % 2], events=events)
        else:
            queued.append(r.render_nosync(g, cam, mode, out=outs[k % 2], events=events))

    for c in cams:                       # sizes the pair workspace for every camera
        r.render(g, c, mode)
    for w in range(warmup):
        frame(w)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for k in range(steps):
        frame(k)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    evs = [ss.StageEvents(dev) for _ in range(steps)]
    torch.cuda.synchronize()
    for k in range(steps):
        frame(k, evs[k])
    torch.cuda.synchronize()
    stages = {s: statistics.mean(e.stage_ms()[s] for e in evs) for s in ss.STAGES}
    frame_ev = statistics.mean(sum(e.stage_ms().values()) for e in evs)
    if not all(q.ok() for q in queued):
        raise RuntimeError("a frame did not fit its pair workspace")
    return ms, stages, frame_ev


def stage_roofline_ms(stages_bytes, blend_slots):
    """Roofline time of each stage: algorithmic bytes at 8 TB/s, the blend's
    issue slots at the FP32 VALU rate."""
    out = {k: b / (PEAK_HBM_GBS * 1e9) * 1e3 for k, b in stages_bytes.items()}
    out["blend"] = blend_slots / (PEAK_VALU_TOPS * 1e12) * 1e3
    return out


def frame_bytes(n, v, p, tiles, width, height):
    passes = (int(math.ceil(math.log2(max(tiles, 2)))) + 7) // 8
    # the colour kernel runs beside the depth order .. ranges (a second
    # stream), so it has no stage of its own; its bytes count in the roofline
    # sum only
    return {"preprocess": n * PRE_BYTES_PER_G,
            "colour": n * COLOUR_BYTES_PER_G + v * COLOUR_BYTES_PER_VISIBLE,
            "depth_order": n * DEPTH_ORDER_BYTES_PER_SLOT + v * DEPTH_ORDER_BYTES_PER_VISIBLE,
            "scan": v * SCAN_BYTES_PER_VISIBLE,
            "emit": v * EMIT_BYTES_PER_VISIBLE + p * EMIT_BYTES_PER_PAIR,
            "sort": p * SORT_BYTES_PER_PAIR_PASS * passes,
            "ranges": p * RANGES_BYTES_PER_PAIR + tiles * RANGES_BYTES_PER_TILE}


def band_bench(ss, g, cams, steps, warmup, n_bands=8):
    """The benchmark frame split into n_bands bands of tile rows, as n_bands
    GPUs would render it (ss_render_band: every Gaussian preprocessed, only
    the band's tiles rendered), each band timed one by one on this GPU with
    stage events: the per-band ms, the slowest band (the split frame's
    critical path, before the image gather) and the per-stage times of the
    middle band."""
    import numpy as np
    cam0 = cams[0]
    bounds = np.linspace(0, cam0.tiles_y, n_bands + 1).round().astype(int)
    r = ss.Renderer(g.device)
    res = {"workload": f"the AccuTile benchmark frame split into {n_bands} bands of tile rows "
                       f"{bounds.tolist()}, each rendered alone over the 8 cameras",
           "band_ms": []}
    for b, (b0, b1) in enumerate(zip(bounds[:-1], bounds[1:])):
        ms, st, _ = time_frames(ss, r, g, cams, "accutile", steps, warmup,
                                band=(int(b0), int(b1 - b0)))
        res["band_ms"].append(round(ms, 4))
        if b == n_bands // 2:
            res["middle_band_stage_ms"] = {k: round(v, 4) for k, v in st.items()}
    res["slowest_band_ms"] = max(res["band_ms"])
    log(f"bands: {res}")
    return res


def pruning_demo(ss, dev, iters=3000):
    """The pruning schedule of Sec. 4.2.2-4.2.3 (80 % soft prunes at 20/30/40 %
    of training, 30 % hard prunes every 10 % from 50 %), scaled to `iters`
    iterations, on a synthetic fit-to-target run through the autograd
    function: a 300k-Gaussian model fitted with Adam and an L1 loss to eight
    800x520 views of a different 100k-Gaussian scene.  Scores are summed over
    the eight views before each prune; the Adam moments are compacted with
    the parameters.  After each prune: Gaussians, render FPS at the training
    resolution and PSNR over the views."""
    import torch

    import scenegen
    from paper_2412_00578_amd import prune as pr
    cams = scenegen.orbit_cameras(8, 12.0, 10.0, 800, 520)
    gt = ss.Gaussians.from_scene(scenegen.scene_blobs(100_000, 60), dev)
    rgt = ss.Renderer(dev)
    targets = [rgt.render(gt, c, "accutile").clone() for c in cams]
    sc = scenegen.scene_blobs(300_000, 61)
    op = torch.tensor(sc.opacity).clamp(1e-4, 1 - 1e-4)
    raw = [torch.tensor(sc.means), torch.tensor(sc.scales).log(), torch.tensor(sc.quats),
           torch.log(op / (1 - op)), torch.tensor(sc.sh)]
    params = [t.to(dev).requires_grad_(True) for t in raw]
    lrs = (1e-3, 5e-3, 1e-3, 5e-2, 2.5e-3)

    def make_opt(ps):
        return torch.optim.Adam([{"params": [p], "lr": lr} for p, lr in zip(ps, lrs)], eps=1e-15)

    opt = make_opt(params)
    act = lambda ps: ss.Gaussians(ps[0].detach(), ps[1].detach().exp(), ps[2].detach(),
                                  torch.sigmoid(ps[3].detach()), ps[4].detach(), 3)

    def measure():
        g = act(params)
        r = ss.Renderer(dev)
        mse = 0.0
        for c, tgt in zip(cams, targets):
            mse += float(((r.render(g, c, "accutile") - tgt) ** 2).mean()) / len(cams)
        for c in cams:
            r.render(g, c, "accutile")
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for k in range(16):
            r.render(g, cams[k % len(cams)], "accutile")
        b.record()
        torch.cuda.synchronize()
        return {"gaussians": g.n, "fps": round(16000.0 / a.elapsed_time(b), 1),
                "psnr_db": round(-10.0 * math.log10(max(mse, 1e-12)), 2)}

    events = {it: (ratio, kind) for it, ratio, kind in pr.Schedule(total=iters).events()}
    log_rows = [dict(iteration=0, kind="start", ratio=0.0, **measure())]
    t0 = time.perf_counter()
    for it in range(iters):
        if it in events:
            ratio, kind = events[it]
            g = act(params)
            score = sum(ss.pruning_score(g, c, "accutile") for c in cams)
            keep = pr.select(score, ratio)
            packed = pr.gather(ss.Gaussians(*[p.detach() for p in params], 3), keep)
            state = [opt.state[p] for p in params]
            moments = {m: pr.gather(ss.Gaussians(*[st[m] for st in state], 3), keep)
                       for m in ("exp_avg", "exp_avg_sq")}
            steps = [st["step"] for st in state]
            fields = ("means", "scales", "quats", "opacity", "sh")
            params = [getattr(packed, f).reshape((-1,) + tuple(p.shape[1:])).requires_grad_(True)
                      for f, p in zip(fields, params)]
            opt = make_opt(params)
            for k, p in enumerate(params):
                opt.state[p] = {"step": steps[k],
                                "exp_avg": getattr(moments["exp_avg"], fields[k]).reshape(p.shape),
                                "exp_avg_sq": getattr(moments["exp_avg_sq"],
                                                      fields[k]).reshape(p.shape)}
            row = dict(iteration=it, kind=kind, ratio=ratio, **measure())
            log_rows.append(row)
            log(f"prune: {row}")
        k = it % len(cams)
        img = ss.render(params[0], params[1].exp(), params[2], torch.sigmoid(params[3]),
                        params[4], cams[k], "accutile")
        loss = (img - targets[k]).abs().mean()
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
    log_rows.append(dict(iteration=iters, kind="end", ratio=0.0, **measure()))
    return {"workload": f"fit of a 300k-Gaussian SH-3 model to eight 800x520 AccuTile views of a "
                        f"100k-Gaussian scene, Adam, L1 loss, {iters} iterations, the paper's "
                        f"schedule scaled by {iters}/30000",
            "train_s": round(time.perf_counter() - t0, 1), "after_each_prune": log_rows}


def c2_bench(ss, dev, modes, warmup):
    """The 150k-Gaussian scene over 64 random orbit cameras, frames one by one:
    ms per frame and the cost per Gaussian-tile pair and per evaluated
    pixel-Gaussian pair."""
    import scenegen
    sc = scenegen.scene_c2()
    cams = scenegen.cameras_c2(64)
    g = ss.Gaussians.from_scene(sc, dev)
    r = ss.Renderer(dev)
    out = {"workload": "150k-Gaussian SH-3 clustered scene (higher opacity, larger scales), "
                       "1600x1040, 64 random orbit cameras, frames one by one"}
    for mode in modes:
        P, V, E, I = work_counters(ss, g, cams, mode)
        ms, stages, _ = time_frames(ss, r, g, cams, mode, len(cams), warmup)
        p, e = statistics.mean(P), statistics.mean(E)
        out[mode] = {"ms_per_frame": round(ms, 4), "fps": round(1000.0 / ms, 1),
                     "stage_ms": {k: round(v, 4) for k, v in stages.items()},
                     "pairs_per_frame": int(p), "evaluated_pairs_per_frame": int(e),
                     "ps_per_pair": round(ms * 1e9 / p, 2),
                     "blend_ps_per_evaluated_pair": round(stages["blend"] * 1e9 / e, 3)}
        log(f"C2 {mode}: {ms:.3f} ms/frame, {out[mode]['ps_per_pair']} ps per Gaussian-tile "
            f"pair, blend {out[mode]['blend_ps_per_evaluated_pair']} ps per evaluated pair")
    return out


def c3_bench(ss, dev, steps, warmup):
    """Differentiable render of the 1M-Gaussian scene at 1264x832: AccuTile
    forward, L1 loss against a seeded target, backward to the means,
    log-scales, quaternions, opacity logits and SH through the autograd
    function, per step."""
    import torch

    import scenegen
    sc = scenegen.scene_c3()
    cam = scenegen.camera_c3()
    means = torch.tensor(sc.means, device=dev, requires_grad=True)
    log_s = torch.tensor(sc.scales, device=dev).log().requires_grad_(True)
    quats = torch.tensor(sc.quats, device=dev, requires_grad=True)
    op = torch.tensor(sc.opacity, device=dev).clamp(1e-6, 1 - 1e-6)
    logits = torch.log(op / (1 - op)).requires_grad_(True)
    sh = torch.tensor(sc.sh, device=dev, requires_grad=True)
    gen = torch.Generator(device=dev).manual_seed(3)
    target = torch.rand((3, cam.height, cam.width), generator=gen, device=dev)
    params = (means, log_s, quats, logits, sh)

    def step():
        for p in params:
            p.grad = None
        img = ss.render(means, log_s.exp(), quats, torch.sigmoid(logits), sh, cam, "accutile")
        loss = (img - target).abs().mean()
        loss.backward()
        return loss

    for _ in range(warmup):
        step()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(steps):
        loss = step()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    res = {"workload": "1M-Gaussian SH-3 clustered scene, 1264x832, AccuTile, L1 loss against a "
                       "seeded U[0,1] target, gradients to means, log-scales, quaternions, opacity "
                       "logits and SH through the autograd function",
           "ms_per_step": round(ms, 4), "steps_per_s": round(1000.0 / ms, 1),
           "loss": round(float(loss.item()), 6)}
    log(f"C3 forward+backward: {res}")
    return res


def backward_bench(ss, g, cams, steps, warmup):
    """The adjoint of the AccuTile frame (blend backward + preprocess backward)
    for a seeded image gradient, with and without the pruning score; each
    kernel timed by the events the library records inside the call."""
    import torch
    dev = g.device
    r = ss.Renderer(dev)
    out = r.render(g, cams[0], "accutile", full=True)
    gen = torch.Generator(device=dev).manual_seed(7)
    dl = torch.randn(out.image.shape, generator=gen, device=dev, dtype=torch.float32)
    res = {}
    for name, score in (("backward", False), ("backward_with_score", True)):
        for _ in range(warmup):
            ss.backward(g, cams[0], out, dl, want_score=score)
        evs = [ss.BackwardEvents(dev) for _ in range(steps)]
        torch.cuda.synchronize()
        for k in range(steps):
            ss.backward(g, cams[0], out, dl, want_score=score, events=evs[k])
        torch.cuda.synchronize()
        parts = {key: statistics.mean(e.ms()[key] for e in evs) for key in evs[0].ms()}
        res[name + "_ms"] = round(sum(parts.values()), 4)
        if not score:
            res["kernel_ms"] = {k: round(v, 4) for k, v in parts.items()}
    walked = int(out.frame.n_last.to(torch.int64).sum().item())
    n, v = g.n, out.n_visible
    t7 = res["kernel_ms"]["blend_bwd"] * 1e-3
    t8 = res["kernel_ms"]["preprocess_bwd"] * 1e-3
    a7 = walked * RATED_SLOTS_PER_WALKED / t7 / 1e12
    b8 = n * PBWD_BYTES_PER_G + v * PBWD_BYTES_PER_VISIBLE
    res["blended_entries_walked"] = walked
    res["roofline"] = {
        "blend_bwd": {"bound": "alu", "achieved": round(a7, 3), "peak": round(PEAK_VALU_TOPS, 1),
                      "unit": "T slots/s", "frac": round(a7 / PEAK_VALU_TOPS, 4),
                      "work": f"{walked} list entries walked back x {RATED_SLOTS_PER_WALKED} "
                              f"slots"},
        "preprocess_bwd": {"bound": "hbm", "achieved": round(b8 / t8 / 1e9, 1),
                           "peak": PEAK_HBM_GBS, "unit": "GB/s",
                           "frac": round(b8 / t8 / 1e9 / PEAK_HBM_GBS, 4),
                           "work": f"{n} Gaussians x {PBWD_BYTES_PER_G} B + {v} with tiles x "
                                   f"{PBWD_BYTES_PER_VISIBLE} B"}}
    res["workload"] = ("adjoint of one AccuTile frame of the 1.5M-Gaussian scene (camera 0), "
                       "seeded N(0,1) image gradient")
    log(f"backward: {res}")
    return res


def serving_bench(ss, dev, scale=1.0, n_sat=400, n_req=2000, n_warm=200, max_batch=8,
                  pool_gib=4):
    """Continuous-batching serving over 4 resident scenes (0.3M / 1M / 3M / 6M
    Gaussians, SH-3, clustered) with random orbit cameras at 640x480,
    1280x720, 1600x1040 or 1920x1080: AccuTile's saturation rate X (every
    request waiting from the start), then p50/p99 latency of Poisson arrivals
    at 0.5X and 0.8X (n_req requests after n_warm warm-up requests), for
    AccuTile and for 3-sigma at the same request rates."""
    import scenegen
    from paper_2412_00578_amd.serve import Request, serve
    t0 = time.perf_counter()
    gs = []
    for k in range(4):
        sc = scenegen.scene_c4(k, scale=scale)
        gs.append(ss.Gaussians.from_scene(sc, dev))
        del sc
    n_res = sum(g.n for g in gs)
    log(f"serving: {n_res} resident Gaussians ({sum(g.nbytes for g in gs) / 2**30:.2f} GiB) "
        f"in {time.perf_counter() - t0:.1f} s")

    def stream(n, qps, seed):
        return [Request(k, s, cam, t) for k, (t, s, cam) in
                enumerate(scenegen.request_stream(n, qps, 4, seed))]

    kw = dict(device=dev, pool_bytes=int(pool_gib * 2**30), max_batch=max_batch)
    out = {"workload": "4 resident scenes 0.3M/1M/3M/6M Gaussians SH-3; cameras on a radius-12 "
                       "orbit; resolutions 640x480/1280x720/1600x1040/1920x1080 uniform; "
                       f"pool {pool_gib} GiB, batches <= {max_batch}, 2 launch slots; "
                       f"{n_req} Poisson requests after {n_warm} warm-up at each rate",
           "resident_gaussians": n_res}
    for mode in ("accutile", "3sigma"):
        serve(gs, stream(60, 1e9, 45), mode=mode, **kw)          # warm-up
        sat = serve(gs, stream(n_sat, 1e9, 46), mode=mode, **kw)
        out[f"saturation_{mode}"] = sat.summary()
        log(f"serving saturation, {mode}: {sat.fps:.1f} requests/s, {sat.summary()}")
        if mode == "accutile":
            X = sat.fps
        for frac in (0.5, 0.8):
            reqs = stream(n_warm + n_req, frac * X, 44)
            st = serve(gs, reqs, mode=mode, skip=n_warm, **kw)
            out[f"poisson_{frac}X_{mode}"] = dict(st.summary(), qps=round(frac * X, 2))
            log(f"serving {mode} at {frac}X = {frac * X:.1f} qps: {st.summary()}")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1_500_000)
    ap.add_argument("--modes", default=",".join(MODES))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 150k-scene, differentiable-render and adjoint measurements")
    ap.add_argument("--serve-scale", type=float, default=1.0,
                    help="scale of the resident scenes of the serving measurement")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only measure the adjoint of the AccuTile frame (for profiling it)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy 5 times (the reference "
                         "kernel for scaling HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2412_00578_amd as ss
    import scenegen

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": a.numel() * 4, "copies": 5}), flush=True)
        return
    t0 = time.perf_counter()
    scene = scenegen.scene_c1(n=args.n)
    cams = scenegen.cameras_c1(8)
    g = ss.Gaussians.from_scene(scene, dev)
    log(f"scene: {scene.n} Gaussians, generated and uploaded in {time.perf_counter() - t0:.1f} s")
    if args.adjoint_only:
        res = backward_bench(ss, g, cams, args.steps, args.warmup)
        print(json.dumps({"backward": res}), flush=True)
        return
    r = ss.Renderer(dev)
    modes = [m for m in args.modes.split(",") if m]
    tiles = cams[0].tiles_x * cams[0].tiles_y

    work = {}
    for mode in modes:
        work[mode] = work_counters(ss, g, cams, mode)
        P, V, E, I = work[mode]
        log(f"{mode}: pairs/frame {np.mean(P):.0f}, evaluated pairs/frame {np.mean(E):.3e}, "
            f"blended pairs/frame {np.mean(I):.3e}, Gaussians with tiles {np.mean(V):.0f}")

    results = {}
    for mode in modes:
        ms, stages, frame_ev = time_frames(ss, r, g, cams, mode, args.steps, args.warmup)
        ms_sync, stages_sync, _ = time_frames(ss, r, g, cams, mode, args.steps, args.warmup,
                                              sync=True)
        P, V, E, I = work[mode]
        steps_cam = [k % len(cams) for k in range(args.steps)]
        p_mean = statistics.mean(P[c] for c in steps_cam)
        e_mean = statistics.mean(E[c] for c in steps_cam)
        v_mean = statistics.mean(V[c] for c in steps_cam)
        i_mean = statistics.mean(I[c] for c in steps_cam)
        rated = e_mean * RATED_SLOTS_PER_EVAL
        counted = e_mean * SLOTS_PER_EVAL + i_mean * SLOTS_PER_BLENDED
        fb = frame_bytes(args.n, v_mean, p_mean, tiles, cams[0].width, cams[0].height)
        roof = stage_roofline_ms(fb, rated)
        results[mode] = {
            "fps": round(1000.0 / ms, 2), "ms_per_frame": round(ms, 4),
            "stage_ms": {k: round(v, 4) for k, v in stages.items()},
            "ms_per_frame_with_stage_events": round(frame_ev, 4),
            "ms_per_frame_readback": round(ms_sync, 4),
            "stage_ms_readback": {k: round(v, 4) for k, v in stages_sync.items()},
            "pairs_per_frame": int(p_mean), "evaluated_pairs_per_frame": int(e_mean),
            "blended_pairs_per_frame": int(i_mean), "gaussians_with_tiles": int(v_mean),
            "blend_rated_tslots": round(rated / (stages["blend"] * 1e-3) / 1e12, 3),
            "blend_counted_tslots": round(counted / (stages["blend"] * 1e-3) / 1e12, 3),
            "stage_gbs": {k: round(fb[k] / (stages[k] * 1e-3) / 1e9, 1) for k in fb
                          if k in stages},
            "stage_roofline_ms": {k: round(v, 4) for k, v in roof.items()},
            "frame_roofline_frac": round(sum(roof.values()) / ms, 4),
        }
        # The same frames as one sequence (Renderer.render_many): the host runs
        # ahead, so the pair-count read-back leaves the GPU idle no longer, and
        # consecutive frames' stages overlap on three streams.
        outs = [torch.empty((3, cams[0].height, cams[0].width), dtype=torch.float32, device=dev)
                for _ in range(2)]
        seq = [cams[k % len(cams)] for k in range(args.steps)]
        r.render_many(g, seq[:args.warmup], mode, outs=[outs[k % 2] for k in range(args.warmup)])
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        r.render_many(g, seq, mode, outs=[outs[k % 2] for k in range(args.steps)])
        stop.record()
        torch.cuda.synchronize()
        ms_pipe = start.elapsed_time(stop) / args.steps
        results[mode].update({"fps_pipelined": round(1000.0 / ms_pipe, 2),
                              "ms_per_frame_pipelined": round(ms_pipe, 4)})
        log(f"{mode}: {ms:.3f} ms/frame one by one ({1000 / ms:.1f} FPS; {ms_sync:.3f} with the "
            f"count read-back), {ms_pipe:.3f} ms/frame "
            f"pipelined; stages " + " ".join(f"{k}={v:.3f}" for k, v in stages.items()))
    for mode in modes:
        if "3sigma" in results and mode != "3sigma":
            results[mode]["speedup_vs_3sigma"] = round(
                results["3sigma"]["ms_per_frame"] / results[mode]["ms_per_frame"], 3)
            results[mode]["speedup_vs_3sigma_pipelined"] = round(
                results["3sigma"]["ms_per_frame_pipelined"] /
                results[mode]["ms_per_frame_pipelined"], 3)

    acc = results.get("accutile") or results[modes[-1]]
    blend_ms = acc["stage_ms"]["blend"]
    e_acc, i_acc = acc["evaluated_pairs_per_frame"], acc["blended_pairs_per_frame"]
    achieved = e_acc * RATED_SLOTS_PER_EVAL / (blend_ms * 1e-3) / 1e12
    counted = (e_acc * SLOTS_PER_EVAL + i_acc * SLOTS_PER_BLENDED) / (blend_ms * 1e-3) / 1e12
    line = {
        "metric": METRIC,
        "value": acc["fps"],
        "unit": "FPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": acc["ms_per_frame"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1.5M-Gaussian SH-3 clustered scene, 1600x1040, 16x16 tiles, "
                               "8 orbit cameras, AccuTile forward render, frames one by one",
                   "n_gaussians": args.n, "width": 1600, "height": 1040, "tile_mode": "accutile"},
        "speedup_vs_3sigma": acc.get("speedup_vs_3sigma"),
        "paper": PAPER,
        "fps_pipelined": acc["fps_pipelined"],
        "frame_roofline_frac": acc["frame_roofline_frac"],
        "modes": results,
        "roofline": {"bound": "alu", "kernel": "blend (k_blend)",
                     "achieved": round(achieved, 3), "peak": round(PEAK_VALU_TOPS, 1),
                     "unit": "T VALU issue slots/s (FP32 lane-op rate)",
                     "frac": round(achieved / PEAK_VALU_TOPS, 4),
                     "traffic": blend_traffic(),
                     "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated; "
                                     "profiles/forward_c1_hbm_traffic.txt)",
                     "work": f"{e_acc} evaluated pixel-Gaussian pairs x {RATED_SLOTS_PER_EVAL} "
                             f"slots per launch",
                     "counted": {"achieved": round(counted, 3),
                                 "frac": round(counted / PEAK_VALU_TOPS, 4),
                                 "work": f"{e_acc} evaluated pairs x {SLOTS_PER_EVAL} slots + "
                                         f"{i_acc} blended pairs x {SLOTS_PER_BLENDED} slots"},
                     "avg_launch_ms": round(blend_ms, 4)},
    }
    if not args.no_extra:
        line["backward"] = backward_bench(ss, g, cams, max(args.steps // 3, 5), args.warmup)
        line["bands_8"] = band_bench(ss, g, cams, max(args.steps // 3, 5), args.warmup)
        line["c2_150k_64_cameras"] = c2_bench(ss, dev, modes, args.warmup)
        line["c3_forward_backward"] = c3_bench(ss, dev, max(args.steps // 3, 5), args.warmup)
        line["pruning"] = pruning_demo(ss, dev)
    if not args.no_serve:
        line["serving"] = serving_bench(ss, dev, args.serve_scale)
        line["serving_p50_ms"] = line["serving"]["poisson_0.8X_accutile"]["p50_ms"]
        line["serving_p99_ms"] = line["serving"]["poisson_0.8X_accutile"]["p99_ms"]
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(scene, cams[0])
        line["cpu_baseline_all_cores"] = cpu_baseline_all_cores(scene, cams[0])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

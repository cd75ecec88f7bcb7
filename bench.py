#!/usr/bin/env python3
"""Forward-render benchmark on one MI355X.

Workload: a 1.5M-Gaussian SH-degree-3 clustered scene (200 anisotropic blobs
plus 10% uniform background in a 20-unit box) rendered at 1600x1040 with 16x16
tiles from 8 orbit cameras (radius 12, 10 degrees elevation), all synthetic and
seeded.  One step is one forward render of one frame: preprocess, depth
order, scan, pair count read-back, key emission, tile sort, tile ranges and
blend.  Each of the three tile assignments (3-sigma, SnugBox, AccuTile) is
timed over the same steps on the same scene twice: frame by frame with
per-stage events (the host waits for each frame's pair count), and as one
sequence (Renderer.render_many): the host runs ahead, and consecutive frames'
preprocess, depth order and blend overlap on three streams, which is how a
fly-through or video renderer runs; `value` is the AccuTile frame rate of the
latter, `fps_sequential` the former.

Per-stage kernel times come from hipEvents the library records on its stream
inside every timed frame.  The blend (the dominant kernel) is reported against
the FP32 VALU roofline; the HBM-bound stages against 8 TB/s.  The CPU baseline
is the test oracle (plain C, one thread) rendering one frame of the same
workload.

A serving measurement follows (see serving_bench): p50/p99 request latency
at 0.5 and 0.8 of the saturation request rate over four resident scenes.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline] [--no-serve]
"""
from __future__ import annotations

import argparse
import hashlib
import json
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
# FP32 operations per evaluated (pixel, Gaussian) pair of the blend's inclusion
# test q = fma(dy, fma(c, dy, (2b) dx), (a dx) dx) <= t: dx, dy, a dx,
# (a dx) dx, (2b) dx, two FMAs and the compare (an FMA counts as one); and per
# blended pair: the exponent scale, exp, sigma * exp, the 0.99 clamp, 1 - alpha,
# T (1 - alpha), alpha T, the stop compare and three colour FMAs.
OPS_PER_EVAL = 8
OPS_PER_CONTRIB = 11
# Algorithmic HBM bytes: the geometry kernel reads 44 B (mean, scale,
# quaternion, opacity) and writes 56 B (geom, conic, count, depth key, tile
# set) per Gaussian, the colour kernel reads the count and writes rgb (20 B) per
# Gaussian and reads the mean and the SH-3 row (204 B) of each Gaussian with
# tiles; the depth order moves 8 B per slot in its compacting first pass plus
# 100 B per Gaussian with tiles over all four passes (keys, values, and the
# last pass's gather of the tile sets into depth order); the tile sort moves
# 20 B per pair per 8-bit pass.
PRE_BYTES_PER_G, PRE_BYTES_PER_VISIBLE = 44 + 56 + 20, 204
DEPTH_ORDER_BYTES_PER_SLOT, DEPTH_ORDER_BYTES_PER_VISIBLE = 8, 100
SORT_BYTES_PER_PAIR_PASS = 20


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


def cpu_baseline(scene, cam, runs=3):
    """The oracle (plain C, single thread) rendering one AccuTile frame."""
    import oracle
    oracle.lib()
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        oracle.render(scene, cam, "accutile")
        times.append(time.perf_counter() - t0)
        log(f"  cpu oracle frame: {times[-1]:.2f} s")
    ms = statistics.median(times) * 1e3
    return {"value": round(1000.0 / ms, 4), "unit": "FPS", "cores": 1, "kind": "oracle",
            "sample": f"one full 1600x1040 AccuTile frame of the 1.5M-Gaussian scene "
                      f"(camera 0), median of {runs} runs, {ms:.0f} ms/frame, "
                      f"on {cpu_model()} ({os.cpu_count()} visible cores)"}


def backward_bench(ss, g, cams, steps, warmup):
    """The adjoint of the AccuTile frame (blend backward + preprocess backward)
    for a seeded image gradient, with and without the pruning score, timed with
    events around ss_render_backward.  Forward state is rendered untimed."""
    import torch
    dev = g.device
    r = ss.Renderer(dev)
    outs = [r.render(g, c, "accutile", full=True) for c in cams[:1]]
    out = outs[0]
    gen = torch.Generator(device=dev).manual_seed(7)
    dl = torch.randn(out.image.shape, generator=gen, device=dev, dtype=torch.float32)
    res = {}
    for name, score in (("backward", False), ("backward_with_score", True)):
        for _ in range(warmup):
            ss.backward(g, cams[0], out, dl, want_score=score)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(steps):
            ss.backward(g, cams[0], out, dl, want_score=score)
        b.record()
        torch.cuda.synchronize()
        res[name + "_ms"] = round(a.elapsed_time(b) / steps, 4)
    n_last = out.frame.n_last.to(torch.int64)
    res["blended_entries_walked"] = int(n_last.sum().item())   # per-pixel list entries walked back
    res["workload"] = ("adjoint of one AccuTile frame of the benchmark scene (camera 0), "
                       "seeded N(0,1) image gradient")
    log(f"backward: {res}")
    return res


def serving_bench(ss, dev, scale=1.0, n_sat=400, n_req=1000, max_batch=8, pool_gib=16):
    """Continuous-batching serving over 4 resident scenes (0.3M / 1M / 3M / 6M
    Gaussians, SH-3, clustered) with random orbit cameras at 640x480,
    1280x720, 1600x1040 or 1920x1080: the saturation rate X (every request
    waiting from the start), then p50/p99 latency at Poisson arrivals of 0.5X
    and 0.8X."""
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
    serve(gs, stream(60, 1e9, 45), mode="accutile", **kw)          # warm-up
    sat = serve(gs, stream(n_sat, 1e9, 46), mode="accutile", **kw)
    X = sat.fps
    out = {"workload": "4 resident scenes 0.3M/1M/3M/6M Gaussians SH-3; cameras on a radius-12 "
                       "orbit; resolutions 640x480/1280x720/1600x1040/1920x1080 uniform; "
                       f"pool {pool_gib} GiB, batches <= {max_batch}, 2 launch slots",
           "resident_gaussians": n_res, "saturation": sat.summary()}
    log(f"serving saturation: {X:.1f} requests/s, {sat.summary()}")
    for frac in (0.5, 0.8):
        st = serve(gs, stream(n_req, frac * X, 44), mode="accutile", **kw)
        out[f"poisson_{frac}X"] = dict(st.summary(), qps=round(frac * X, 2))
        log(f"serving at {frac}X = {frac * X:.1f} qps: {st.summary()}")
    s3 = serve(gs, stream(n_sat, 1e9, 46), mode="3sigma", **kw)
    out["saturation_3sigma"] = s3.summary()
    log(f"serving saturation, 3-sigma: {s3.summary()}")
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
    ap.add_argument("--serve-scale", type=float, default=1.0,
                    help="scale of the resident scenes of the serving measurement")
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
    r = ss.Renderer(dev)
    r_stats = ss.Renderer(dev, stats=True)
    modes = [m for m in args.modes.split(",") if m]

    # Work counters per camera (untimed): pairs and evaluated pixel-Gaussian pairs.
    work = {}
    for mode in modes:
        P, E, V, I = [], [], [], []
        for cam in cams:
            out = r_stats.render(g, cam, mode, full=True)
            torch.cuda.synchronize()
            P.append(out.n_pairs)
            V.append(out.n_visible)
            E.append(int(out.frame.n_eval.to(torch.int64).sum().item()))
            I.append(int(out.frame.n_contrib.to(torch.int64).sum().item()))
        work[mode] = (P, E, V, I)
        log(f"{mode}: pairs/frame {np.mean(P):.0f}, evaluated pairs/frame {np.mean(E):.3e}, "
            f"blended pairs/frame {np.mean(I):.3e}, Gaussians with tiles {np.mean(V):.0f}")
    del r_stats

    results = {}
    for mode in modes:
        for w in range(args.warmup):
            r.render(g, cams[w % len(cams)], mode)
        evs = [ss.StageEvents(dev) for _ in range(args.steps)]
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        for k in range(args.steps):
            r.render(g, cams[k % len(cams)], mode, events=evs[k])
        stop.record()
        torch.cuda.synchronize()
        total_ms = start.elapsed_time(stop)
        ms = total_ms / args.steps
        stages = {s: statistics.mean(e.stage_ms()[s] for e in evs) for s in ss.STAGES}
        P, E, V, I = work[mode]
        steps_cam = [k % len(cams) for k in range(args.steps)]
        p_mean = statistics.mean(P[c] for c in steps_cam)
        e_mean = statistics.mean(E[c] for c in steps_cam)
        v_mean = statistics.mean(V[c] for c in steps_cam)
        i_mean = statistics.mean(I[c] for c in steps_cam)
        blend_ops = e_mean * OPS_PER_EVAL + i_mean * OPS_PER_CONTRIB
        passes = (int(np.ceil(np.log2(cams[0].tiles_x * cams[0].tiles_y))) + 7) // 8
        results[mode] = {
            "fps": round(1000.0 / ms, 2), "ms_per_frame": round(ms, 4),
            "stage_ms": {k: round(v, 4) for k, v in stages.items()},
            "pairs_per_frame": int(p_mean), "evaluated_pairs_per_frame": int(e_mean),
            "blended_pairs_per_frame": int(i_mean), "gaussians_with_tiles": int(v_mean),
            "blend_ops_per_frame": int(blend_ops),
            "blend_tops": round(blend_ops / (stages["blend"] * 1e-3) / 1e12, 3),
            "preprocess_gbs": round((args.n * PRE_BYTES_PER_G + v_mean * PRE_BYTES_PER_VISIBLE) /
                                    (stages["preprocess"] * 1e-3) / 1e9,
                                    1),
            "depth_order_gbs": round((args.n * DEPTH_ORDER_BYTES_PER_SLOT +
                                      v_mean * DEPTH_ORDER_BYTES_PER_VISIBLE) /
                                     (stages["depth_order"] * 1e-3) / 1e9, 1),
            "sort_gbs": round(p_mean * SORT_BYTES_PER_PAIR_PASS * passes /
                              (stages["sort"] * 1e-3) / 1e9, 1),
        }
        # The same frames as one sequence (Renderer.render_many): the host runs
        # ahead, so the pair-count read-back leaves the GPU idle no longer, and
        # consecutive frames' stages overlap on three streams.
        outs = [torch.empty((3, cams[0].height, cams[0].width), dtype=torch.float32, device=dev)
                for _ in range(2)]
        seq = [cams[k % len(cams)] for k in range(args.steps)]
        r.render_many(g, seq[:args.warmup], mode, outs=[outs[k % 2] for k in range(args.warmup)])
        torch.cuda.synchronize()
        start.record()
        r.render_many(g, seq, mode, outs=[outs[k % 2] for k in range(args.steps)])
        stop.record()
        torch.cuda.synchronize()
        ms_pipe = start.elapsed_time(stop) / args.steps
        results[mode].update({"fps_sequential": results[mode]["fps"],
                              "ms_per_frame_sequential": results[mode]["ms_per_frame"],
                              "fps": round(1000.0 / ms_pipe, 2),
                              "ms_per_frame": round(ms_pipe, 4)})
        log(f"{mode}: {ms:.3f} ms/frame sequential, {ms_pipe:.3f} ms/frame pipelined "
            f"({1000 / ms_pipe:.1f} FPS); stages "
            + " ".join(f"{k}={v:.3f}" for k, v in stages.items()))

    acc = results.get("accutile") or results[modes[-1]]
    base = results.get("3sigma")
    blend_ms = acc["stage_ms"]["blend"]
    achieved = acc["blend_ops_per_frame"] / (blend_ms * 1e-3) / 1e12
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
                               "8 orbit cameras, AccuTile forward render",
                   "n_gaussians": args.n, "width": 1600, "height": 1040, "tile_mode": "accutile"},
        "speedup_vs_3sigma": round(base["ms_per_frame"] / acc["ms_per_frame"], 3) if base else None,
        "modes": results,
        "roofline": {"bound": "alu", "kernel": "blend (k_blend)",
                     "achieved": round(achieved, 3), "peak": round(PEAK_VALU_TOPS, 1),
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_VALU_TOPS, 4),
                     "traffic": blend_traffic(),
                     "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated; "
                                     "profiles/forward_c1_hbm_traffic.txt)",
                     "work": f"{acc['evaluated_pairs_per_frame']} evaluated pixel-Gaussian pairs "
                             f"x {OPS_PER_EVAL} FP32 ops + {acc['blended_pairs_per_frame']} "
                             f"blended pairs x {OPS_PER_CONTRIB} FP32 ops per launch",
                     "avg_launch_ms": round(blend_ms, 4)},
    }
    line["backward"] = backward_bench(ss, g, cams, max(args.steps // 3, 5), args.warmup)
    if not args.no_serve:
        line["serving"] = serving_bench(ss, dev, args.serve_scale)
        line["serving_p50_ms"] = line["serving"]["poisson_0.8X"]["p50_ms"]
        line["serving_p99_ms"] = line["serving"]["poisson_0.8X"]["p99_ms"]
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(scene, cams[0])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

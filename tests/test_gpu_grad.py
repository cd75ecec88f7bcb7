"""GPU adjoint (ss_render_backward) against the FP64 gradient oracle.

The oracle is the dense FP64 renderer of oracle/grad.py, pinned by finite
differences, with its masks taken from the FP32 tiled oracle (the decisions
the GPU forward makes).  Pixels whose stop decision exp rounding could flip
get a zero upstream gradient.  Per parameter group the GPU gradient must have
relative L2 error <= 1e-4 and cosine >= 0.99999 against the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from oracle import grad as og

pytestmark = pytest.mark.gpu
GROUPS = ("means", "scales", "quats", "opacity", "sh")


@pytest.fixture(scope="module")
def ss():
    import paper_2412_00578_amd as ss
    ss.lib()
    return ss


def _oracle_grad_linear(scene, cam, pixels, weights, fr):
    """FP64 autograd of sum(weights * C) w.r.t. the linear parameters."""
    f = lambda a: torch.tensor(np.asarray(a, np.float64), dtype=og.DT, requires_grad=True)
    leaves = {"means": f(scene.means), "scales": f(scene.scales), "quats": f(scene.quats),
              "opacity": f(scene.opacity), "sh": f(scene.sh)}
    rec = og.records64(leaves["means"], leaves["scales"], leaves["quats"], leaves["opacity"],
                       leaves["sh"], scene.sh_degree, cam)
    order = oracle.depth_order(fr.records)
    incl = og.masks_from_tiled(fr, cam, order, pixels)
    C = og.blend_masked(rec, torch.as_tensor(order), pixels, incl, cam.bg)
    (C * torch.as_tensor(weights, dtype=og.DT)).sum().backward()
    return {k: v.grad.numpy() for k, v in leaves.items()}


def _compare(got, want, tag=""):
    for k in GROUPS:
        a = np.asarray(got[k], np.float64).ravel()
        b = np.asarray(want[k], np.float64).ravel()
        nb = np.linalg.norm(b)
        rel = np.linalg.norm(a - b) / max(nb, 1e-30)
        cos = float(a @ b / max(np.linalg.norm(a) * nb, 1e-300))
        print(f"[grad{tag}] {k:8s} |ref|={nb:.3e} rel_l2={rel:.2e} cos={cos:.8f}", flush=True)
        assert rel <= 1e-4, (k, rel)
        assert cos >= 0.99999, (k, cos)


def _weights(cam, fr, seed):
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((3, cam.height, cam.width))
    w[:, fr.ambiguous] = 0.0
    return w


def test_backward_matches_oracle_small(ss, gpu_device):
    sc, cam = scenegen.scene_c3_fd(), scenegen.camera_fd()
    fr = oracle.render(sc, cam, "accutile")
    w = _weights(cam, fr, 5)
    pix = oracle.all_pixels(cam)
    want = _oracle_grad_linear(sc, cam, pix, w.reshape(3, -1).T, fr)
    g = ss.Gaussians.from_scene(sc, gpu_device)
    out = ss.Renderer(gpu_device).render(g, cam, "accutile", full=True)
    gr = ss.backward(g, cam, out, torch.as_tensor(w, dtype=torch.float32, device=gpu_device))
    torch.cuda.synchronize()
    got = {k: getattr(gr, k).cpu().numpy() for k in GROUPS}
    got["opacity"] = got["opacity"].reshape(-1)
    _compare(got, want)


def test_backward_sh_rows_of_odd_length(ss, gpu_device):
    # 17 stored coefficients per Gaussian (51-float rows): the preprocess
    # adjoint stages SH through LDS; the padding coefficient gets no gradient.
    import dataclasses
    sc, cam = scenegen.scene_c3_fd(), scenegen.camera_fd()
    pad = np.full((sc.n, 1, 3), 0.7, np.float32)
    sc = dataclasses.replace(sc, sh=np.ascontiguousarray(np.concatenate([sc.sh, pad], axis=1)))
    fr = oracle.render(sc, cam, "accutile")
    w = _weights(cam, fr, 6)
    pix = oracle.all_pixels(cam)
    want = _oracle_grad_linear(sc, cam, pix, w.reshape(3, -1).T, fr)
    g = ss.Gaussians.from_scene(sc, gpu_device)
    out = ss.Renderer(gpu_device).render(g, cam, "accutile", full=True)
    gr = ss.backward(g, cam, out, torch.as_tensor(w, dtype=torch.float32, device=gpu_device))
    torch.cuda.synchronize()
    got = {k: getattr(gr, k).cpu().numpy() for k in GROUPS}
    got["opacity"] = got["opacity"].reshape(-1)
    assert np.all(got["sh"][:, 16, :] == 0.0)
    _compare(got, want)


def test_backward_into_misaligned_sh_gradient(ss, gpu_device):
    # dL/dh written into a view 4 bytes past a 16-byte boundary: the adjoint
    # takes its scalar-store path and must give the same gradients.
    sc, cam = scenegen.scene_c3_fd(), scenegen.camera_fd()
    g = ss.Gaussians.from_scene(sc, gpu_device)
    out = ss.Renderer(gpu_device).render(g, cam, "accutile", full=True)
    w = torch.as_tensor(np.random.default_rng(8).standard_normal((3, cam.height, cam.width)),
                        dtype=torch.float32, device=gpu_device)
    ref = ss.backward(g, cam, out, w)
    buf = torch.zeros(g.sh.numel() + 4, dtype=torch.float32, device=gpu_device)
    view = buf[1:1 + g.sh.numel()].view(g.sh.shape)
    assert view.data_ptr() % 16 == 4
    got = ss.backward(g, cam, out, w, sh_out=view)
    torch.cuda.synchronize()
    # the per-Gaussian sums are atomics, so two runs agree to rounding only
    for k in ("sh", "means"):
        a, b = getattr(got, k).double(), getattr(ref, k).double()
        assert float((a - b).norm() / b.norm()) <= 1e-6, k
    assert float(buf[0]) == 0.0 and float(buf[-3]) == 0.0


def test_autograd_function_l1_loss(ss, gpu_device):
    # torch autograd through the activations: scales = exp(log_s), opacity = sigmoid(logit).
    sc, cam = scenegen.scene_c3_fd(), scenegen.camera_fd()
    rng = np.random.default_rng(9)
    target = rng.uniform(0, 1, (3, cam.height, cam.width)).astype(np.float32)
    dev = gpu_device
    t = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev, requires_grad=True)
    means, log_s, quats, logits, sh = (t(sc.means), t(sc.log_scales), t(sc.quats), t(sc.logits),
                                       t(sc.sh))
    scales, opac = torch.exp(log_s), torch.sigmoid(logits)
    # the oracle's forward decisions come from the very FP32 values the GPU renders
    sc.scales = scales.detach().cpu().numpy()
    sc.opacity = opac.detach().cpu().numpy()
    fr = oracle.render(sc, cam, "accutile")
    img = ss.render(means, scales, quats, opac, sh, cam, "accutile")
    tgt = torch.as_tensor(target, device=dev)
    mask = torch.as_tensor(~fr.ambiguous, device=dev)[None]
    loss = (torch.abs(img - tgt) * mask).mean()
    loss.backward()
    # oracle: the same loss; dL/dC = sign(C - target) / (3HW) with the oracle's C
    p = og.Params(sc)
    pix = oracle.all_pixels(cam)
    with torch.no_grad():
        rec = p.records(cam)
    order = oracle.depth_order(fr.records)
    incl = og.masks_from_tiled(fr, cam, order, pix)
    C = og.blend_masked(p.records(cam), torch.as_tensor(order), pix, incl, cam.bg)
    tgt_t = torch.as_tensor(target.reshape(3, -1).T, dtype=og.DT)
    m_t = torch.as_tensor((~fr.ambiguous).reshape(-1, 1), dtype=og.DT)
    L = (torch.abs(C - tgt_t) * m_t).sum() / (3 * cam.height * cam.width)
    L.backward()
    want = {"means": p.means.grad.numpy(), "scales": p.log_scales.grad.numpy(),
            "quats": p.quats.grad.numpy(), "opacity": p.logits.grad.numpy(),
            "sh": p.sh.grad.numpy()}
    got = {"means": means.grad.cpu().numpy(), "scales": log_s.grad.cpu().numpy(),
           "quats": quats.grad.cpu().numpy(), "opacity": logits.grad.cpu().numpy(),
           "sh": sh.grad.cpu().numpy()}
    # residual signs must agree for the comparison to be meaningful
    gimg = img.detach().cpu().numpy().reshape(3, -1).T
    Cn = C.detach().numpy()
    same = np.sign(gimg - target.reshape(3, -1).T) == np.sign(Cn - target.reshape(3, -1).T)
    assert same.mean() > 0.9999
    _compare(got, want, "-l1")


def test_pruning_score_matches_oracle(ss, gpu_device):
    sc, cam = scenegen.scene_c3_fd(), scenegen.camera_fd()
    fr = oracle.render(sc, cam, "accutile")
    pix = oracle.all_pixels(cam)
    order = oracle.depth_order(fr.records)
    incl = og.masks_from_tiled(fr, cam, order, pix)
    p = og.Params(sc)
    with torch.no_grad():
        rec = p.records(cam)
    # dC/dg with g = exp(-q/2) held as an explicit leaf per (pixel, Gaussian)
    q = og._q(rec, torch.as_tensor(order), pix)
    gval = torch.exp(-0.5 * q).detach().requires_grad_(True)
    sig = rec["sigma"][order][None, :]
    al = torch.where(torch.as_tensor(incl), torch.clamp(sig * gval, max=og.ALPHA_MAX),
                     torch.zeros_like(gval))
    one_m = 1 - al
    T_ex = torch.cumprod(torch.cat([torch.ones_like(one_m[:, :1]), one_m[:, :-1]], 1), 1)
    C = (al * T_ex) @ rec["rgb"][order]
    score = torch.zeros(len(order), dtype=og.DT)
    for ch in range(3):
        (gc,) = torch.autograd.grad(C[:, ch].sum(), gval, retain_graph=True)
        score += (gc * gc).sum(0)
    want = np.zeros(sc.n)
    want[order] = score.numpy()
    g = ss.Gaussians.from_scene(sc, gpu_device)
    got = ss.pruning_score(g, cam, "accutile").cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    print(f"[score] rel_l2={rel:.2e}, nonzero={np.count_nonzero(want)}", flush=True)
    assert rel <= 1e-4
    # ranking agrees on the Gaussians that matter
    top = np.argsort(-want)[:200]
    assert len(set(top) & set(np.argsort(-got)[:200])) >= 195


def test_backward_full_size_masked_tiles(ss, gpu_device):
    # 1M Gaussians, SH-3, 1264x832; the upstream gradient lives on 12 seeded
    # tiles, so the oracle solves one small dense problem per tile.
    sc = scenegen.scene_c3(n=1_000_000)
    cam = scenegen.camera_c3()
    print(f"[case] backward n={sc.n} {cam.width}x{cam.height}", flush=True)
    rng = np.random.default_rng(33)
    fr = oracle.render(sc, cam, "accutile", blend_tiles=None)
    lens = fr.ranges[:, 1] - fr.ranges[:, 0]
    cand = np.nonzero(lens > 50)[0]
    tiles = rng.choice(cand, size=12, replace=False)
    img, tf, nl, amb, ne, _ = oracle.blend(cam, fr.ranges, fr.sorted_values, fr.records, tiles)
    fr.image, fr.t_final, fr.n_last, fr.ambiguous = img, tf, nl, amb
    w = np.zeros((3, cam.height, cam.width))
    for tl in tiles:
        ty, tx = divmod(int(tl), cam.tiles_x)
        blk = rng.standard_normal((3, 16, 16))
        w[:, ty * 16:ty * 16 + 16, tx * 16:tx * 16 + 16] = blk
    w[:, amb] = 0.0
    # oracle, tile by tile, on the Gaussians of each tile's list
    want = {k: np.zeros((sc.n,) + np.shape(getattr(sc, k))[1:]) for k in
            ("means", "scales", "quats", "sh")}
    want["opacity"] = np.zeros(sc.n)
    for tl in tiles:
        ty, tx = divmod(int(tl), cam.tiles_x)
        s, e = fr.ranges[tl]
        ids = np.unique(fr.sorted_values[s:e]).astype(np.int64)
        sub = sc.subset(ids)
        ys, xs = np.mgrid[ty * 16:ty * 16 + 16, tx * 16:tx * 16 + 16]
        pix = np.stack([xs.ravel(), ys.ravel()], 1)
        f = lambda a: torch.tensor(np.asarray(a, np.float64), dtype=og.DT, requires_grad=True)
        L = {"means": f(sub.means), "scales": f(sub.scales), "quats": f(sub.quats),
             "opacity": f(sub.opacity), "sh": f(sub.sh)}
        rec = og.records64(L["means"], L["scales"], L["quats"], L["opacity"], L["sh"], 3, cam)
        loc = {int(g): k for k, g in enumerate(ids)}
        order_g = oracle.depth_order(fr.records)
        in_tile = np.isin(order_g, ids)
        order_local = np.array([loc[int(g)] for g in order_g[in_tile]], np.int64)
        incl_full = og.masks_from_tiled(fr, cam, order_g[in_tile], pix)
        C = og.blend_masked(rec, torch.as_tensor(order_local), pix, incl_full, cam.bg)
        wt = w[:, pix[:, 1], pix[:, 0]].T
        (C * torch.as_tensor(wt, dtype=og.DT)).sum().backward()
        for k in want:
            want[k][ids] += L[k].grad.numpy()
    g = ss.Gaussians.from_scene(sc, gpu_device)
    out = ss.Renderer(gpu_device).render(g, cam, "accutile", full=True)
    gr = ss.backward(g, cam, out, torch.as_tensor(w, dtype=torch.float32, device=gpu_device))
    torch.cuda.synchronize()
    got = {k: getattr(gr, k).cpu().numpy() for k in GROUPS}
    got["opacity"] = got["opacity"].reshape(-1)
    _compare(got, want, "-c3")


def test_backward_through_clamped_stacks(ss, gpu_device):
    """Stacks of near-opaque Gaussians in front of the camera: many pixels see
    alpha clamped at 0.99 or just below it (T_before = T_after / (1 - alpha)
    amplifies the recurrence's rounding by up to 100 per step), mixed with
    moderate ones, until the transmittance stops the walk at 1e-4."""
    rng = np.random.default_rng(77)
    n = 240
    xy = rng.uniform(-0.25, 0.25, size=(n, 2))
    z = rng.uniform(2.0, 3.0, size=n)
    means = np.column_stack([xy, z])
    scales = np.exp(rng.uniform(-2.6, -1.6, size=(n, 3)))
    quats = rng.standard_normal((n, 4))
    kind = rng.integers(0, 3, size=n)
    opac = np.where(kind == 0, rng.uniform(0.995, 0.9999, n),         # clamped at the centre
                    np.where(kind == 1, rng.uniform(0.95, 0.985, n),  # just below the clamp
                             rng.uniform(0.2, 0.6, n)))
    cols = rng.uniform(-0.8, 0.8, size=(n, 3))
    sc = scenegen.fixture_scene(means, scales, quats, opac, cols)
    cam = scenegen.camera_fd()
    fr = oracle.render(sc, cam, "accutile")
    stopped = int((fr.n_last < fr.n_eval).sum())
    print(f"[case] clamped stacks: {stopped} of {fr.n_last.size} pixels stop early", flush=True)
    assert stopped > 500                       # the walk is cut by the transmittance
    w = _weights(cam, fr, 8)
    pix = oracle.all_pixels(cam)
    want = _oracle_grad_linear(sc, cam, pix, w.reshape(3, -1).T, fr)
    g = ss.Gaussians.from_scene(sc, gpu_device)
    out = ss.Renderer(gpu_device).render(g, cam, "accutile", full=True)
    gr = ss.backward(g, cam, out, torch.as_tensor(w, dtype=torch.float32, device=gpu_device))
    torch.cuda.synchronize()
    got = {k: getattr(gr, k).cpu().numpy() for k in GROUPS}
    got["opacity"] = got["opacity"].reshape(-1)
    _compare(got, want, " clamped")

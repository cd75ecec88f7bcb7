"""FP64 dense differentiable renderer (torch, CPU) for gradient checks.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The renderer recomputes the per-Gaussian records in FP64 from the parameters
(the chain of Sec. 3.2.1: camera space, projection, Sigma_3D = R S S^T R^T, EWA
with the FOV-clamped Jacobian and +0.3 dilation, conic, SH colour) and blends
every pixel against all Gaussians in depth order (Eqs. render_alpha,
2d_gaussian_scalar, contribution).  The discrete parts of the forward pass
(which pixel-Gaussian pairs pass q <= t, and where each pixel stops because
the transmittance would drop below 1e-4) enter as constant masks: either
computed here in FP64 (``masks_fp64``) or taken from the FP32 tiled oracle
(``masks_from_tiled``), which makes the same decisions as the GPU.  The
0.99 alpha clamp, the colour clamp at 0 and the Jacobian clamp are
differentiated as the functions they are (zero slope where clamped).

Gradients are torch autograd of this renderer; they are pinned by central
finite differences of the same renderer with masks recomputed per evaluation.
"""
from __future__ import annotations

import math

import numpy as np
import torch

DT = torch.float64
T_MIN = 1e-4
ALPHA_MAX = 0.99


def sh_basis_t(d: torch.Tensor) -> torch.Tensor:
    """Real SH basis (degree <= 3, Condon-Shortley phase) at unit directions
    d [N,3] -> [N,16]."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    c0 = 0.28209479177387814
    c1 = 0.4886025119029199
    c2a, c2b, c2c = 1.0925484305920792, 0.31539156525252005, 0.5462742152960396
    c3a, c3b, c3c = 0.5900435899266435, 2.890611442640554, 0.4570457994644658
    c3d, c3e = 0.3731763325901154, 1.445305721320277
    xx, yy, zz = x * x, y * y, z * z
    return torch.stack([
        torch.full_like(x, c0),
        -c1 * y, c1 * z, -c1 * x,
        c2a * x * y, -c2a * y * z, c2b * (2 * zz - xx - yy), -c2a * x * z, c2c * (xx - yy),
        -c3a * y * (3 * xx - yy), c3b * x * y * z, -c3c * y * (4 * zz - xx - yy),
        c3d * z * (2 * zz - 3 * xx - 3 * yy), -c3c * x * (4 * zz - xx - yy),
        c3e * z * (xx - yy), -c3a * x * (xx - 3 * yy),
    ], dim=1)


def records64(means, scales, quats, opacity, sh, sh_degree, cam):
    """FP64 records from (linear) parameters.  Returns a dict of tensors
    u, v, depth, a, b, c, t, sigma, rgb [N,3]; culled Gaussians are not
    removed here (the masks exclude them)."""
    R = torch.as_tensor(np.asarray(cam.R, np.float64), dtype=DT)
    tc = torch.as_tensor(np.asarray(cam.t, np.float64), dtype=DT)
    pc = means @ R.T + tc
    x, y, z = pc[:, 0], pc[:, 1], pc[:, 2]
    fx, fy, cx, cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    u = fx * x / z + cx
    v = fy * y / z + cy
    qn = quats / quats.norm(dim=1, keepdim=True)
    w, qx, qy, qz = qn[:, 0], qn[:, 1], qn[:, 2], qn[:, 3]
    Rq = torch.stack([
        torch.stack([1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - w * qz), 2 * (qx * qz + w * qy)], -1),
        torch.stack([2 * (qx * qy + w * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - w * qx)], -1),
        torch.stack([2 * (qx * qz - w * qy), 2 * (qy * qz + w * qx), 1 - 2 * (qx * qx + qy * qy)], -1),
    ], dim=1)
    M = Rq * scales[:, None, :]
    S3 = M @ M.transpose(1, 2)
    limx = 1.3 * (0.5 * cam.width / fx)
    limy = 1.3 * (0.5 * cam.height / fy)
    txz = torch.clamp(x / z, -limx, limx)
    tyz = torch.clamp(y / z, -limy, limy)
    zero = torch.zeros_like(z)
    J = torch.stack([torch.stack([fx / z, zero, -fx * txz / z], -1),
                     torch.stack([zero, fy / z, -fy * tyz / z], -1)], dim=1)
    Tm = J @ R
    S2 = Tm @ S3 @ Tm.transpose(1, 2)
    A = S2[:, 0, 0] + 0.3
    B = S2[:, 0, 1]
    C = S2[:, 1, 1] + 0.3
    D = A * C - B * B
    cpos = -(R.T @ tc)
    dvec = means - cpos
    dirn = dvec / dvec.norm(dim=1, keepdim=True)
    nb = (sh_degree + 1) ** 2
    Y = sh_basis_t(dirn)[:, :nb]
    rgb = torch.clamp(torch.einsum("nk,nkc->nc", Y, sh[:, :nb, :]) + 0.5, min=0.0)
    t = 2.0 * torch.log(255.0 * opacity)
    return {"u": u, "v": v, "depth": z, "a": C / D, "b": -B / D, "c": A / D, "t": t,
            "sigma": opacity, "rgb": rgb, "D": D}


def _q(rec, order, pixels):
    px = torch.as_tensor(pixels[:, 0] + 0.5, dtype=DT)[:, None]
    py = torch.as_tensor(pixels[:, 1] + 0.5, dtype=DT)[:, None]
    dx = px - rec["u"][order][None, :]
    dy = py - rec["v"][order][None, :]
    return (rec["a"][order][None, :] * dx * dx + 2.0 * rec["b"][order][None, :] * dx * dy
            + rec["c"][order][None, :] * dy * dy)


def blend_masked(rec, order, pixels, incl, bg=(0.0, 0.0, 0.0)):
    """Colours [P,3] for pixels [P,2] with the Gaussians `order` (front to back)
    and the constant contribution mask incl [P, len(order)]."""
    q = _q(rec, order, pixels)
    incl_t = torch.as_tensor(incl, dtype=torch.bool)
    al = torch.clamp(rec["sigma"][order][None, :] * torch.exp(-0.5 * q), max=ALPHA_MAX)
    al = torch.where(incl_t, al, torch.zeros_like(al))
    one_m = 1.0 - al
    T_excl = torch.cumprod(torch.cat([torch.ones_like(one_m[:, :1]), one_m[:, :-1]], dim=1), dim=1)
    w = al * T_excl
    col = w @ rec["rgb"][order]
    T_fin = T_excl[:, -1] * one_m[:, -1] if one_m.shape[1] else torch.ones(len(pixels), dtype=DT)
    return col + T_fin[:, None] * torch.as_tensor(bg, dtype=DT)[None, :]


def masks_fp64(rec, order, pixels):
    """The forward pass's decisions in FP64: include iff q <= t, stop before the
    first included Gaussian that would take T below 1e-4.  Returns (incl,
    signature) where the signature also records the alpha clamp states."""
    with torch.no_grad():
        q = _q(rec, order, pixels)
        t = rec["t"][order][None, :]
        valid = (rec["D"][order] > 0)[None, :] & (rec["depth"][order] > 0)[None, :]
        pas = (q <= t) & valid
        a_raw = rec["sigma"][order][None, :] * torch.exp(-0.5 * q)
        al = torch.where(pas, torch.clamp(a_raw, max=ALPHA_MAX), torch.zeros_like(q))
        T_excl = torch.cumprod(torch.cat([torch.ones_like(al[:, :1]), (1 - al)[:, :-1]], 1), 1)
        stop_here = pas & (T_excl * (1 - al) < T_MIN)
        after = torch.cumsum(stop_here.to(torch.int32), dim=1) > 0
        incl = pas & ~after
        clamped = incl & (a_raw > ALPHA_MAX)
    return incl.numpy(), (incl.numpy(), clamped.numpy())


def masks_from_tiled(fr, cam, order, pixels):
    """Contribution masks from the tiled oracle frame `fr` (the decisions the
    GPU makes): Gaussian i contributes at pixel p iff it sits in p's tile list
    before n_last and passes the q <= t test, q the record's quadratic form in
    FP64 at the pixel centre."""
    pos = {int(g): k for k, g in enumerate(order)}
    incl = np.zeros((len(pixels), len(order)), bool)
    geom, conic = fr.records.geom, fr.records.conic
    for r, (px, py) in enumerate(pixels):
        tile = (py // 16) * cam.tiles_x + (px // 16)
        s, e = fr.ranges[tile]
        nl = int(fr.n_last[py, px])
        fxp, fyp = px + 0.5, py + 0.5
        for j in range(s, s + nl):
            i = int(fr.sorted_values[j])
            dx = fxp - float(geom[i, 0])
            dy = fyp - float(geom[i, 1])
            a, b, c = (float(x) for x in conic[i, :3])
            qq = (a * dx * dx + c * dy * dy) + 2.0 * b * dx * dy
            if qq <= float(geom[i, 3]):
                incl[r, pos[i]] = True
    return incl


class Params:
    """Pre-activation parameters as FP64 leaves: means, log-scales, quaternions,
    opacity logits, SH coefficients."""

    def __init__(self, scene):
        f = lambda a: torch.tensor(np.asarray(a, np.float64), dtype=DT, requires_grad=True)
        self.means = f(scene.means)
        self.log_scales = f(scene.log_scales if scene.log_scales is not None
                            else np.log(scene.scales))
        self.quats = f(scene.quats)
        op = np.asarray(scene.opacity, np.float64)
        self.logits = f(scene.logits if scene.logits is not None else np.log(op / (1 - op)))
        self.sh = f(scene.sh)
        self.sh_degree = scene.sh_degree

    def leaves(self):
        return [self.means, self.log_scales, self.quats, self.logits, self.sh]

    def names(self):
        return ["means", "log_scales", "quats", "logits", "sh"]

    def records(self, cam):
        return records64(self.means, torch.exp(self.log_scales), self.quats,
                         torch.sigmoid(self.logits), self.sh, self.sh_degree, cam)


def depth_order64(rec) -> np.ndarray:
    with torch.no_grad():
        z = rec["depth"].numpy()
        ok = (z > 0.2) & (rec["D"].numpy() > 0)
    idx = np.nonzero(ok)[0]
    return idx[np.argsort(z[idx], kind="stable")]


def grad_weighted(params: Params, cam, pixels, weights, incl=None, order=None):
    """Autograd gradient of L = sum(weights * C) [weights: P x 3] with the masks
    held constant.  Returns (L, {name: grad ndarray})."""
    for p in params.leaves():
        p.grad = None
    rec = params.records(cam)
    if order is None:
        order = depth_order64(rec)
    if incl is None:
        incl, _ = masks_fp64(rec, order, pixels)
    C = blend_masked(rec, torch.as_tensor(order), pixels, incl, cam.bg)
    L = (C * torch.as_tensor(weights, dtype=DT)).sum()
    L.backward()
    return float(L.detach()), {n: p.grad.numpy().copy() for n, p in zip(params.names(), params.leaves())}


def loss_fd(params: Params, cam, pixels, weights, order):
    """L and the decision signature with masks recomputed in FP64 (no grad)."""
    with torch.no_grad():
        rec = params.records(cam)
        o = torch.as_tensor(order)
        incl, sig = masks_fp64(rec, o, pixels)
        C = blend_masked(rec, o, pixels, incl, cam.bg)
        rgb_clamp = (rec["rgb"] == 0).numpy()
        L = float((C * torch.as_tensor(weights, dtype=DT)).sum())
    return L, (sig, rgb_clamp)


def same_signature(s1, s2) -> bool:
    (a1, b1), c1 = s1
    (a2, b2), c2 = s2
    return np.array_equal(a1, a2) and np.array_equal(b1, b2) and np.array_equal(c1, c2)


def gaussian_pixels(rec, i, cam, pad=2.0):
    """Pixels inside Gaussian i's (padded) 1/255 box: the only pixels whose
    colour a small change of its parameters can move."""
    with torch.no_grad():
        a, b, c, t = (float(rec[k][i]) for k in ("a", "b", "c", "t"))
        u, v = float(rec["u"][i]), float(rec["v"][i])
    det = a * c - b * b
    if t <= 0 or det <= 0:
        return np.zeros((0, 2), np.int64)
    hx, hy = math.sqrt(t * c / det) + pad, math.sqrt(t * a / det) + pad
    x0, x1 = max(0, int(math.floor(u - hx))), min(cam.width - 1, int(math.ceil(u + hx)))
    y0, y1 = max(0, int(math.floor(v - hy))), min(cam.height - 1, int(math.ceil(v + hy)))
    if x0 > x1 or y0 > y1:
        return np.zeros((0, 2), np.int64)
    ys, xs = np.mgrid[y0:y1 + 1, x0:x1 + 1]
    return np.stack([xs.ravel(), ys.ravel()], 1)

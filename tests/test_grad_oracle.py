"""Pins of the gradient oracle (oracle/grad.py).

The dense FP64 renderer must reproduce the C oracle's records and image, and
its autograd gradient must equal central finite differences (masks recomputed
per evaluation; parameters whose perturbation changes a discrete decision are
skipped and counted)."""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from oracle import grad as og


def test_torch_sh_basis_matches_c_oracle():
    rng = np.random.default_rng(1)
    d = rng.standard_normal((50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    got = og.sh_basis_t(torch.as_tensor(d)).numpy()
    want = np.stack([oracle.sh_basis(v) for v in d])
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13)


def test_fp64_records_match_c_oracle():
    sc = scenegen.scene_c3_fd()
    cam = scenegen.camera_fd()
    rec32 = oracle.preprocess(sc, cam, "accutile")
    p = og.Params(sc)
    with torch.no_grad():
        r = p.records(cam)
    ok = rec32.conic[:, 0] != 0
    assert ok.sum() > 1500
    np.testing.assert_allclose(r["u"].numpy()[ok], rec32.geom[ok, 0], rtol=1e-6, atol=1e-4)
    np.testing.assert_allclose(r["v"].numpy()[ok], rec32.geom[ok, 1], rtol=1e-6, atol=1e-4)
    for k, col in (("a", 0), ("b", 1), ("c", 2)):
        ref = rec32.conic[ok, col].astype(np.float64)
        scale = np.abs(rec32.conic[ok, :3]).max(axis=1)
        assert np.all(np.abs(r[k].numpy()[ok] - ref) <= 1e-5 * scale + 1e-12)
    np.testing.assert_allclose(r["rgb"].numpy()[ok], rec32.rgb[ok, :3], rtol=1e-5, atol=1e-5)


def test_masked_dense_blend_reproduces_tiled_image():
    sc = scenegen.scene_c3_fd()
    cam = scenegen.camera_fd()
    fr = oracle.render(sc, cam, "accutile")
    p = og.Params(sc)
    with torch.no_grad():
        rec = p.records(cam)
    order = oracle.depth_order(fr.records)
    pix = oracle.all_pixels(cam)
    incl = og.masks_from_tiled(fr, cam, order, pix)
    with torch.no_grad():
        C = og.blend_masked(rec, torch.as_tensor(order), pix, incl).numpy()
    got = fr.image.reshape(3, -1).T
    ok = ~fr.ambiguous.reshape(-1)
    assert np.abs(C[ok] - got[ok]).max() <= 2e-5


@pytest.mark.slow
def test_autograd_equals_finite_differences():
    sc = scenegen.scene_c3_fd()
    cam = scenegen.camera_fd()
    p = og.Params(sc)
    pix = oracle.all_pixels(cam)
    rng = np.random.default_rng(3)
    weights = rng.standard_normal((len(pix), 3))
    _, g = og.grad_weighted(p, cam, pix, weights)
    with torch.no_grad():
        rec = p.records(cam)
    order = og.depth_order64(rec)
    visible = [i for i in order if len(og.gaussian_pixels(rec, i, cam)) > 0]
    leaves = dict(zip(p.names(), p.leaves()))
    checked = skipped = 0
    worst = 0.0
    for k in range(150):
        i = int(visible[rng.integers(len(visible))])
        name = ["means", "log_scales", "quats", "logits", "sh"][k % 5]
        leaf = leaves[name]
        sub = tuple(int(rng.integers(s)) for s in leaf.shape[1:])
        idx = (i,) + sub
        pix_i = og.gaussian_pixels(rec, i, cam)
        w_i = weights[pix_i[:, 1] * cam.width + pix_i[:, 0]]
        base_L, base_sig = og.loss_fd(p, cam, pix_i, w_i, order)
        theta = float(leaf.detach()[idx])
        h = 1e-6 * max(1.0, abs(theta))
        vals = []
        sigs = []
        for s in (+1, -1):
            with torch.no_grad():
                leaf[idx] = theta + s * h
            with torch.no_grad():
                o2 = og.depth_order64(p.records(cam))
            L, sig = og.loss_fd(p, cam, pix_i, w_i, order)
            vals.append(L)
            sigs.append(og.same_signature(sig, base_sig) and np.array_equal(o2, order))
        with torch.no_grad():
            leaf[idx] = theta
        if not all(sigs):
            skipped += 1
            continue
        fd = (vals[0] - vals[1]) / (2 * h)
        an = float(g[name][idx])
        err = abs(fd - an) / (max(1.0, abs(fd)))
        worst = max(worst, err)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (name, idx, fd, an)
        checked += 1
    assert checked >= 120, (checked, skipped)
    print(f"checked {checked}, skipped {skipped}, worst relative error {worst:.2e}")


def _fma64_exact(a, b, c):
    """Correctly rounded FP64 value of a*b + c: exact rational arithmetic, then
    CPython's correctly rounded integer division."""
    from fractions import Fraction
    x = Fraction(a) * Fraction(b) + Fraction(c)
    return x.numerator / x.denominator


def test_inclusion_band_covers_faithful_fp64_orders():
    """The blend's inclusion-ambiguity band: the quadratic form of an FP32
    record, q = a dx^2 + 2b dx dy + c dy^2 with dx, dy FP64 offsets of an FP32
    pixel centre, evaluated in FP64 in any order with at most four roundings
    per term, lies within gamma_4 * S of the exact q (S = the sum of the terms'
    magnitudes, gamma_4 = 4v/(1-4v), v = 2^-53).  Checked against exact
    rationals for the oracle's unfused order and for a fused multiply-add
    order, on random forms (including needle-like, ill-conditioned ones) and
    on thresholds placed just outside the band, where both orders must decide
    as the exact q does."""
    from fractions import Fraction as F
    v = 2.0 ** -53
    gam = 4 * v / (1 - 4 * v)
    rng = np.random.default_rng(12)
    worst = 0.0
    for k in range(3000):
        a, c = np.abs(rng.standard_normal(2)).astype(np.float32) * np.float32(rng.choice([1e-3, 0.1, 3]))
        rho = rng.choice([rng.uniform(-0.99, 0.99), 1.0 - 10.0 ** -rng.uniform(3, 7)])
        b = np.float32(rho * np.sqrt(float(a) * float(c)))
        u, vv = (rng.uniform(-50, 1650, 2)).astype(np.float32)
        px, py = rng.integers(0, 1600, 2)
        dx, dy = (px + 0.5) - float(u), (py + 0.5) - float(vv)   # exact in FP64
        A, B, C = float(a), float(b), float(c)
        q_o = (A * dx * dx + C * dy * dy) + 2.0 * B * dx * dy
        q_f = _fma64_exact(_fma64_exact(C, dy, (2.0 * B) * dx), dy, (A * dx) * dx)
        exact = F(A) * F(dx) ** 2 + 2 * F(B) * F(dx) * F(dy) + F(C) * F(dy) ** 2
        S = abs(F(A)) * F(dx) ** 2 + 2 * abs(F(B) * F(dx) * F(dy)) + abs(F(C)) * F(dy) ** 2
        for q in (q_o, q_f):
            err = abs(F(q) - exact)
            assert err <= F(gam) * S, (k, a, b, c, dx, dy, q)
            if S > 0:
                worst = max(worst, float(err / S) / v)
        t_in = float(exact) + 2.01 * gam * float(S)
        t_out = float(exact) - 2.01 * gam * float(S)
        if F(t_in) - exact > F(gam) * S:
            assert q_o <= t_in and q_f <= t_in
        if exact - F(t_out) > F(gam) * S:
            assert not (q_o <= t_out) and not (q_f <= t_out)
    print(f"worst |fl(q) - q| / S = {worst:.2f} ulp64 (bound {gam / v:.2f})")


def test_oracle_flags_a_pixel_on_the_inclusion_threshold():
    """A record whose q equals t exactly at one pixel centre (a = t, b = 0,
    the centre one pixel right of the mean) is flagged ambiguous there, and
    pixels far from the ellipse boundary are not."""
    import oracle
    import scenegen
    cam = scenegen.Camera(16, 16, 16.0, 16.0, 8.0, 8.0, np.eye(3), np.zeros(3))
    t = np.float32(2.0 * np.log(255.0 * 0.5))
    rec = oracle.Records(geom=np.array([[7.5, 7.5, 3.0, t]], np.float32),
                         conic=np.array([[t, 0.0, 1.0, 0.5]], np.float32),
                         rgb=np.array([[1.0, 1.0, 1.0, 0.0]], np.float32),
                         counts=np.array([1], np.uint32), mode=2, visible=1)
    ranges = np.array([[0, 1]], np.uint32)
    img, tf, nl, amb, ne, nc = oracle.blend(cam, ranges, np.array([0], np.uint32), rec)
    # pixel (8, 7): centre (8.5, 7.5), dx = 1, dy = 0, q = t exactly
    assert amb[7, 8] and amb[7, 6]
    assert not amb[7, 7] and not amb[0, 0] and not amb[15, 15]
    assert amb.sum() < 16



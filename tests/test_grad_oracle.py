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


def _fma32_exact(a, b, c):
    """Correctly rounded (to nearest, ties to even) FP32 value of a*b + c,
    from exact rational arithmetic."""
    from fractions import Fraction
    x = Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c))
    guess = np.float32(float(x))
    cands = [np.nextafter(guess, np.float32(-np.inf)), guess,
             np.nextafter(guess, np.float32(np.inf))]
    best = min(cands, key=lambda v: (abs(Fraction(float(v)) - x),
                                     int(np.array(v).view(np.int32)) & 1))
    return np.float32(best)


def test_fma32_is_correctly_rounded():
    """The FP32 fused multiply-add of the gradient oracle against exact rational
    rounding and against the C library's fmaf, including near-cancellation and
    exact-tie inputs."""
    import ctypes
    import ctypes.util
    libm = ctypes.CDLL(ctypes.util.find_library("m"))
    libm.fmaf.argtypes = [ctypes.c_float] * 3
    libm.fmaf.restype = ctypes.c_float
    rng = np.random.default_rng(12)
    cases = []
    for _ in range(3000):
        a, b = rng.standard_normal(2).astype(np.float32) * np.float32(rng.choice([1e-3, 1, 1e3]))
        c = np.float32(-(np.float64(a) * np.float64(b)) * (1 + rng.standard_normal() * 1e-6))
        cases.append((a, b, c))                                  # near cancellation
        cases.append((a, b, np.float32(rng.standard_normal() * 10)))
    # a*b + c exactly halfway between two FP32 values (ties to even)
    cases.append((np.float32(1 + 2 ** -12), np.float32(1 + 2 ** -12), np.float32(-1.0)))
    cases.append((np.float32(1.0), np.float32(2 ** -24), np.float32(1.0)))
    cases.append((np.float32(1.0), np.float32(3 * 2 ** -24), np.float32(1.0)))
    for a, b, c in cases:
        got = og.fma32(a, b, c)
        assert got == _fma32_exact(a, b, c), (a, b, c)
        assert got == np.float32(libm.fmaf(float(a), float(b), float(c))), (a, b, c)

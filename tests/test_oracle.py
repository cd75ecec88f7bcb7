"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed forms,
invariants, library routines for single steps (scipy rotations and spherical
harmonics, numpy eigenvalues and sorts), brute force (the exact tile predicate
TILE*, exact rationals, per-pixel blending over all Gaussians) and the paper's
own equations for the SnugBox extremes.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.special import sph_harm_y

import oracle
import scenegen
from oracle import brute

F32 = np.float32


def single(mean, scale, quat=(1, 0, 0, 0), opacity=0.9, colour=(1.0, 0.5, 0.25)):
    return scenegen.fixture_scene([mean], [scale], [quat], [opacity], [colour])


def cam_c0():
    return scenegen.camera_c0()


# ------------------------------------------------------------ projection / EWA

def test_projection_known_point():
    # x=1, y=2, z=4 with f=256, c=128: u = 256*1/4 + 128 = 192, v = 256*2/4 + 128 = 256.
    rec = oracle.preprocess(single((1.0, 2.0, 4.0), (0.05,) * 3), cam_c0(), "3sigma")
    assert rec.geom[0, 0] == F32(192.0) and rec.geom[0, 1] == F32(256.0)
    assert rec.geom[0, 2] == F32(4.0)


def test_on_axis_isotropic_closed_form():
    # Isotropic s on the optical axis: Sigma_2D = (f s / z)^2 I + 0.3 I, so the
    # conic is 1/((f s/z)^2 + 0.3) on the diagonal and 0 off it.
    for s, z in [(0.01, 3.0), (0.05, 4.0), (0.2, 5.5)]:
        rec = oracle.preprocess(single((0.0, 0.0, z), (s, s, s)), cam_c0(), "3sigma")
        var = (256.0 * float(F32(s)) / z) ** 2 + 0.3
        a, b, c = rec.conic[0, :3]
        assert a == pytest.approx(1.0 / var, rel=2e-7)
        assert c == pytest.approx(1.0 / var, rel=2e-7)
        assert abs(b) <= 1e-7 * a
        assert rec.geom[0, 0] == F32(128.0) and rec.geom[0, 1] == F32(128.0)


def test_isotropic_is_rotation_invariant():
    rng = np.random.default_rng(5)
    base = None
    for _ in range(6):
        q = rng.standard_normal(4)
        rec = oracle.preprocess(single((0.3, -0.2, 3.0), (0.04,) * 3, q / np.linalg.norm(q)),
                                cam_c0(), "3sigma")
        if base is None:
            base = rec.conic[0, :3].astype(np.float64)
        np.testing.assert_allclose(rec.conic[0, :3], base, rtol=1e-6, atol=1e-9)


def test_quaternion_sign_and_norm_do_not_matter():
    rng = np.random.default_rng(6)
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    r1 = oracle.preprocess(single((0.1, 0.2, 3.0), (0.02, 0.05, 0.01), q), cam_c0(), "3sigma")
    r2 = oracle.preprocess(single((0.1, 0.2, 3.0), (0.02, 0.05, 0.01), -q), cam_c0(), "3sigma")
    r3 = oracle.preprocess(single((0.1, 0.2, 3.0), (0.02, 0.05, 0.01), 2.0 * q), cam_c0(),
                           "3sigma")
    assert np.array_equal(r1.conic, r2.conic) and np.array_equal(r1.geom, r2.geom)
    np.testing.assert_allclose(r3.conic, r1.conic, rtol=1e-6)


def _ewa_reference(mean, scale, quat, cam):
    """Independent FP64 EWA: scipy rotation, Jacobian by central differences."""
    R = np.asarray(cam.R, np.float64)
    t = np.asarray(cam.t, np.float64)
    w, x, y, z = (float(v) for v in quat)
    Rq = Rotation.from_quat([x, y, z, w]).as_matrix()
    S3 = Rq @ np.diag(np.asarray(scale, np.float64) ** 2) @ Rq.T
    pc = R @ np.asarray(mean, np.float64) + t

    def proj(p):
        return np.array([cam.fx * p[0] / p[2] + cam.cx, cam.fy * p[1] / p[2] + cam.cy])

    J = np.zeros((2, 3))
    for k in range(3):
        h = 1e-6 * max(1.0, abs(pc[k]))
        e = np.zeros(3)
        e[k] = h
        J[:, k] = (proj(pc + e) - proj(pc - e)) / (2 * h)
    S2 = J @ R @ S3 @ R.T @ J.T + 0.3 * np.eye(2)
    return np.linalg.inv(S2), proj(pc)


def test_ewa_matches_independent_jacobian():
    rng = np.random.default_rng(7)
    cam = scenegen.orbit_cameras(8, 12.0, 10.0, 320, 240)[3]
    for _ in range(40):
        mean = rng.uniform(-2, 2, 3)
        scale = np.exp(rng.normal(-2.5, 0.7, 3)).astype(F32)
        q = rng.standard_normal(4)
        q = (q / np.linalg.norm(q)).astype(F32)
        sc = single(mean, scale, q)
        rec = oracle.preprocess(sc, cam, "3sigma")
        conic, uv = _ewa_reference(sc.means[0], sc.scales[0], sc.quats[0], cam)
        # keep means well inside the field of view, where the Jacobian clamp is inactive
        if not (0 < uv[0] < cam.width and 0 < uv[1] < cam.height) or rec.conic[0, 0] == 0:
            continue
        np.testing.assert_allclose(rec.geom[0, :2], uv, rtol=1e-6)
        got = np.array([[rec.conic[0, 0], rec.conic[0, 1]], [rec.conic[0, 1], rec.conic[0, 2]]])
        np.testing.assert_allclose(got, conic, rtol=2e-6, atol=1e-6 * np.abs(conic).max())


def test_fov_clamp_of_the_jacobian():
    # Off-screen means: J is evaluated at x/z, y/z clamped to 1.3 times the
    # half-FOV tangent (W/2)/fx, (H/2)/fy; inside the limit nothing changes.
    cam = scenegen.Camera(200, 100, 100.0, 100.0, 100.0, 50.0, np.eye(3), np.zeros(3))
    limx, limy = 1.3 * 1.0, 1.3 * 0.5
    rng = np.random.default_rng(17)
    for _ in range(20):
        z = rng.uniform(2.0, 6.0)
        q = rng.standard_normal(4)
        q = (q / np.linalg.norm(q)).astype(F32)
        s = np.exp(rng.normal(-2.0, 0.5, 3)).astype(F32)
        for fx_, fy_ in [(0.9 * limx, -0.8 * limy), (2.5 * limx, 0.3 * limy),
                         (-0.2 * limx, -3.0 * limy), (-4.0 * limx, 2.0 * limy)]:
            sc = single((fx_ * z, fy_ * z, z), s, q)
            rec = oracle.preprocess(sc, cam, "3sigma")
            m = sc.means[0].astype(np.float64)
            cx_, cy_ = np.clip(m[0] / m[2], -limx, limx), np.clip(m[1] / m[2], -limy, limy)
            conic, _ = _ewa_reference((cx_ * m[2], cy_ * m[2], m[2]), sc.scales[0], sc.quats[0],
                                      cam)
            got = np.array([[rec.conic[0, 0], rec.conic[0, 1]], [rec.conic[0, 1],
                                                                   rec.conic[0, 2]]])
            np.testing.assert_allclose(got, conic, rtol=2e-6, atol=1e-6 * np.abs(conic).max())


def test_near_plane_and_nonfinite_cull():
    sc = scenegen.fixture_scene(
        [(0, 0, 0.1), (0, 0, -3), (np.nan, 0, 3), (0, 0, 3), (0, 0, 3)],
        [(0.05,) * 3, (0.05,) * 3, (0.05,) * 3, (0.05, np.inf, 0.05), (0.05,) * 3],
        [(1, 0, 0, 0)] * 4 + [(0, 0, 0, 0)], [0.5] * 5, [(0.5, 0.5, 0.5)] * 5)
    for mode in oracle.MODES:
        rec = oracle.preprocess(sc, cam_c0(), mode)
        assert rec.visible == 0 and rec.counts.sum() == 0
        assert not rec.geom.any() and not rec.conic.any()


# ------------------------------------------------------------ threshold / colour

def test_threshold_defines_alpha_cutoff():
    # Sec. 4.1: q = t is exactly where alpha = sigma exp(-q/2) = 1/255.
    for sig in [0.01, 0.1, 0.35, 0.5, 0.99]:
        rec = oracle.preprocess(single((0, 0, 3.0), (0.05,) * 3, opacity=sig), cam_c0(), "3sigma")
        t = float(rec.geom[0, 3])
        assert float(F32(sig)) * math.exp(-t / 2) == pytest.approx(1 / 255, rel=1e-6)


def test_low_opacity_culled_only_with_opacity_aware_modes():
    sc = single((0, 0, 3.0), (0.05,) * 3, opacity=1.0 / 260.0)
    assert oracle.preprocess(sc, cam_c0(), "3sigma").counts[0] > 0
    for mode in ("snugbox", "accutile"):
        rec = oracle.preprocess(sc, cam_c0(), mode)
        assert rec.counts[0] == 0 and rec.visible == 0


def _real_sh_textbook(l, m, d):
    """Real SH from scipy's complex Y_l^m (Condon-Shortley phase included)."""
    x, y, z = d
    theta = math.acos(max(-1.0, min(1.0, z)))
    phi = math.atan2(y, x)
    if m == 0:
        return sph_harm_y(l, 0, theta, phi).real
    Y = sph_harm_y(l, abs(m), theta, phi)
    return math.sqrt(2.0) * (Y.real if m > 0 else Y.imag)


def test_sh_basis_matches_scipy():
    rng = np.random.default_rng(8)
    for _ in range(25):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        got = oracle.sh_basis(d)
        want = [_real_sh_textbook(l, m, d) for l in range(4) for m in range(-l, l + 1)]
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def test_sh_basis_orthonormal():
    # Monte-Carlo quadrature over the sphere: the Gram matrix is the identity.
    rng = np.random.default_rng(9)
    d = rng.standard_normal((200000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = np.stack([oracle.sh_basis(v) for v in d[:20000]])
    G = Y.T @ Y * (4 * np.pi / len(Y))
    np.testing.assert_allclose(G, np.eye(16), atol=0.08)


def test_sh_degree0_colour():
    h0 = np.array([0.7, -0.3, 2.0])
    rec = oracle.preprocess(single((0.2, 0.1, 3.0), (0.05,) * 3, colour=h0), cam_c0(), "3sigma")
    want = np.maximum(0.0, 0.28209479177387814 * h0 + 0.5)
    np.testing.assert_allclose(rec.rgb[0, :3], want, rtol=1e-7)


# ------------------------------------------------------------ tile assignment

def _records(scene, cam, mode):
    return oracle.preprocess(scene, cam, mode)


def test_3sigma_radius_matches_eigvalsh():
    rec = _records(scenegen.scene_c0(n=2000), cam_c0(), "3sigma")
    checked = 0
    for i in np.nonzero(rec.conic[:, 0])[0]:
        a, b, c = rec.conic[i, :3].astype(np.float64)
        lam = np.linalg.eigvalsh(np.linalg.inv(np.array([[a, b], [b, c]])))
        lo, hi = lam
        x0, x1, _, _ = oracle.extent(rec.geom[i], rec.conic[i], "3sigma")
        r = (x1 - x0) / 2
        disc = ((hi - lo) / 2) ** 2
        if disc >= 0.1 + 1e-6:
            r_ref = 3.0 * math.sqrt(hi)
            if abs(r_ref - round(r_ref)) > 1e-9:
                assert r == math.ceil(r_ref)
                checked += 1
        else:
            assert r >= math.ceil(3.0 * math.sqrt(hi) - 1e-9)
    assert checked > 100


def test_snugbox_matches_paper_equations_and_sampling():
    # The box from Eqs. ellipse_intersect and bbox_args (solved as printed) and
    # from dense sampling of the boundary agree with the oracle's closed form.
    rec = _records(scenegen.scene_c0(n=600), cam_c0(), "snugbox")
    n = 0
    for i in np.nonzero(rec.conic[:, 0])[0]:
        a, b, c = rec.conic[i, :3].astype(np.float64)
        t = float(rec.geom[i, 3])
        u, v = rec.geom[i, :2].astype(np.float64)
        x0, x1, y0, y1 = oracle.extent(rec.geom[i], rec.conic[i], "snugbox")
        if abs(b) > 1e-12:
            xarg = math.sqrt(-b * b * t / ((b * b - a * c) * a))
            ys = []
            for xd in (xarg, -xarg):
                rad = max(0.0, (b * b - a * c) * xd * xd + t * c)
                ys += [(-b * xd + s * math.sqrt(rad)) / c for s in (1, -1)]
            assert v + max(ys) == pytest.approx(y1, rel=1e-9, abs=1e-9)
            assert v + min(ys) == pytest.approx(y0, rel=1e-9, abs=1e-9)
            yarg = math.sqrt(-b * b * t / ((b * b - a * c) * c))
            xs = []
            for yd in (yarg, -yarg):
                rad = max(0.0, (b * b - a * c) * yd * yd + t * a)
                xs += [(-b * yd + s * math.sqrt(rad)) / a for s in (1, -1)]
            assert u + max(xs) == pytest.approx(x1, rel=1e-9, abs=1e-9)
            assert u + min(xs) == pytest.approx(x0, rel=1e-9, abs=1e-9)
        bx, by = brute.ellipse_boundary(rec.geom[i], rec.conic[i], n=4000)
        w = x1 - x0
        assert bx.max() <= x1 + 1e-9 * (1 + abs(x1)) and bx.max() >= x1 - 1e-3 * w
        assert bx.min() >= x0 - 1e-9 * (1 + abs(x0)) and bx.min() <= x0 + 1e-3 * w
        n += 1
    assert n > 300


def _check_accutile_vs_tilestar(geom, conic, tx_n, ty_n):
    got = set(int(t) for t in oracle.tile_list(geom, conic, "accutile", tx_n, ty_n))
    sure, maybe = brute.tile_star(geom, conic, tx_n, ty_n)
    sure, maybe = set(sure.tolist()), set(maybe.tolist())
    assert sure - maybe <= got, sorted((sure - maybe) - got)
    assert got <= sure | maybe, sorted(got - sure - maybe)
    return got


def test_accutile_equals_tilestar_on_c0():
    cam = cam_c0()
    rec = _records(scenegen.scene_c0(), cam, "accutile")
    n = 0
    for i in np.nonzero(rec.counts)[0]:
        _check_accutile_vs_tilestar(rec.geom[i], rec.conic[i], cam.tiles_x, cam.tiles_y)
        n += 1
    assert n > 9000


def test_accutile_equals_tilestar_random_ellipses():
    rng = np.random.default_rng(11)
    tx_n, ty_n = 24, 18
    for _ in range(3000):
        L = np.diag(np.exp(rng.uniform(0.0, 4.0, 2)))
        th = rng.uniform(0, np.pi)
        Rm = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
        S = Rm @ L @ L @ Rm.T + 0.3 * np.eye(2)
        Q = np.linalg.inv(S)
        sig = rng.uniform(0.01, 1.0)
        geom = np.array([rng.uniform(-40, 16 * tx_n + 40), rng.uniform(-40, 16 * ty_n + 40), 1.0,
                         2 * math.log(255 * sig)], F32)
        conic = np.array([Q[0, 0], Q[0, 1], Q[1, 1], sig], F32)
        if geom[3] <= 0:
            continue
        _check_accutile_vs_tilestar(geom, conic, tx_n, ty_n)


def test_accutile_exact_rational_small_fixtures():
    # Exact rational TILE* on tiny records; includes needles, large ellipses and
    # both iteration directions (rows and columns).
    rng = np.random.default_rng(12)
    tx_n, ty_n = 8, 6
    hits = 0
    for k in range(150):
        a, c = np.exp(rng.uniform(-6, 0, 2))
        b = rng.uniform(-0.95, 0.95) * math.sqrt(a * c)
        geom = np.array([rng.uniform(-10, 138), rng.uniform(-10, 106), 1.0,
                         rng.uniform(0.5, 11.0)], F32)
        conic = np.array([a, b, c, 0.5], F32)
        got = set(int(t) for t in oracle.tile_list(geom, conic, "accutile", tx_n, ty_n))
        want = brute.tile_star_exact(geom, conic, tx_n, ty_n)
        assert got == want, (k, sorted(got ^ want))
        hits += len(want)
    assert hits > 100


def test_accutile_disk_is_circle_rect_test():
    # Isotropic conic a = c, b = 0: the ellipse is a disk of radius sqrt(t/a).
    rng = np.random.default_rng(13)
    for _ in range(300):
        a = float(F32(math.exp(rng.uniform(-6, -1))))
        t = float(F32(rng.uniform(0.5, 11.0)))
        u, v = float(F32(rng.uniform(-20, 150))), float(F32(rng.uniform(-20, 120)))
        geom = np.array([u, v, 1.0, t], F32)
        conic = np.array([a, 0.0, a, 0.5], F32)
        got = set(int(x) for x in oracle.tile_list(geom, conic, "accutile", 8, 7))
        want = brute.disk_tiles(u, v, math.sqrt(t / a), 8, 7)
        sure, maybe = brute.tile_star(geom, conic, 8, 7)
        assert got ^ want <= set(maybe.tolist())


@pytest.mark.parametrize("case", ["1", "2.1", "2.2", "2.3", "3"])
def test_accutile_proof_cases(case):
    """Appendix proof sketch: ellipses built for each case, iterated by rows."""
    # (u, v, semi-axis x, semi-axis y, tilt) in pixels; the tile rows are 16 px.
    specs = {
        "1": (40.0, 40.0, 10.0, 5.0, 0.3),    # fits inside one tile row
        "2.1": (40.0, 30.0, 25.0, 7.0, 0.2),  # crosses one row boundary, x-extremes in row
        "2.2": (40.0, 30.0, 30.0, 12.0, 0.6),  # row holding only y_max
        "2.3": (60.0, 34.0, 40.0, 14.0, 0.5),  # row holding x_min and y_min only
        "3": (64.0, 40.0, 60.0, 22.0, 0.7),   # middle row crossed top and bottom
    }
    u, v, sx, sy, th = specs[case]
    Rm = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    t = 9.0
    S = Rm @ np.diag([sx * sx / t, sy * sy / t]) @ Rm.T
    Q = np.linalg.inv(S)
    geom = np.array([u, v, 1.0, t], F32)
    conic = np.array([Q[0, 0], Q[0, 1], Q[1, 1], 0.5], F32)
    got = set(int(x) for x in oracle.tile_list(geom, conic, "accutile", 12, 8))
    assert got == brute.tile_star_exact(geom, conic, 12, 8)
    snug = set(int(x) for x in oracle.tile_list(geom, conic, "snugbox", 12, 8))
    assert got <= snug


def test_subset_relations_c0_lowsigma():
    # With t <= 9 (sigma <= e^4.5/255) the opacity-aware box lies inside the
    # 3-sigma square, so AccuTile <= SnugBox <= 3-sigma tile sets.
    cam = cam_c0()
    sc = scenegen.scene_c0_lowsigma()
    r3 = _records(sc, cam, "3sigma")
    rs = _records(sc, cam, "snugbox")
    for i in np.nonzero(rs.counts)[0]:
        assert rs.geom[i, 3] <= 9.0
        s3 = set(oracle.tile_list(r3.geom[i], r3.conic[i], "3sigma", cam.tiles_x, cam.tiles_y))
        ss = set(oracle.tile_list(rs.geom[i], rs.conic[i], "snugbox", cam.tiles_x, cam.tiles_y))
        sa = set(oracle.tile_list(rs.geom[i], rs.conic[i], "accutile", cam.tiles_x, cam.tiles_y))
        assert sa <= ss <= s3


def test_snugbox_exceeds_3sigma_only_for_high_opacity():
    # For t > 9 the 1/255 support can reach past 3 standard deviations (the
    # 3-sigma square then drops visible contributions); for t <= 9 never.
    cam = cam_c0()
    sc = scenegen.scene_c0()
    r3 = _records(sc, cam, "3sigma")
    rs = _records(sc, cam, "snugbox")
    outside = 0
    for i in np.nonzero(rs.counts)[0]:
        s3 = set(oracle.tile_list(r3.geom[i], r3.conic[i], "3sigma", cam.tiles_x, cam.tiles_y))
        ss = set(oracle.tile_list(rs.geom[i], rs.conic[i], "snugbox", cam.tiles_x, cam.tiles_y))
        if not ss <= s3:
            assert rs.geom[i, 3] > 9.0
            outside += 1
    assert outside >= 0


# ------------------------------------------------------------ keys / sort / ranges

def test_keys_sort_ranges_textbook():
    cam = cam_c0()
    fr = oracle.render(scenegen.scene_c0(n=3000), cam, "accutile", blend_tiles=None)
    rec = fr.records
    assert fr.n_pairs == int(rec.counts.sum()) == len(fr.keys)
    # every Gaussian's emitted set is its tile set, at its offset
    off = np.concatenate([[0], fr.offsets]).astype(np.int64)
    for i in np.nonzero(rec.counts)[0][:500]:
        tl = oracle.tile_list(rec.geom[i], rec.conic[i], "accutile", cam.tiles_x, cam.tiles_y)
        seg = fr.keys[off[i]:off[i + 1]]
        assert np.array_equal(seg >> np.uint64(32), tl.astype(np.uint64))
        assert np.all(fr.values[off[i]:off[i + 1]] == i)
        assert np.all((seg & np.uint64(0xffffffff)).astype(np.uint32) ==
                      rec.geom[i, 2:3].view(np.uint32)[0])
    order = np.lexsort((fr.values, fr.keys))
    assert np.array_equal(fr.sorted_keys, fr.keys[order])
    assert np.array_equal(fr.sorted_values, fr.values[order])
    tiles = (fr.sorted_keys >> np.uint64(32)).astype(np.int64)
    n_t = cam.tiles_x * cam.tiles_y
    assert np.array_equal(fr.ranges[:, 0], np.searchsorted(tiles, np.arange(n_t), "left"))
    assert np.array_equal(fr.ranges[:, 1], np.searchsorted(tiles, np.arange(n_t), "right"))


def test_emission_order_rows_unless_taller():
    # AccuTile walks rows when the SnugBox tile rectangle has no more rows than
    # columns (ties included), else columns; 3-sigma and SnugBox walk rows.  The
    # emitted tiles are therefore in row-major or column-major order.
    cam = cam_c0()
    for mode in ("3sigma", "snugbox", "accutile"):
        rec = oracle.preprocess(scenegen.scene_c0(n=4000, seed=4, log_s=(-2.5, 0.6)), cam, mode)
        seen = {"rows": 0, "cols": 0}
        for i in np.nonzero(rec.counts > 1)[0]:
            tl = oracle.tile_list(rec.geom[i], rec.conic[i], mode, cam.tiles_x, cam.tiles_y)
            x0, y0, x1, y1 = oracle.tile_rect(rec.geom[i], rec.conic[i], mode, cam.tiles_x,
                                              cam.tiles_y)
            tx, ty = tl % cam.tiles_x, tl // cam.tiles_x
            if mode == "accutile" and (y1 - y0) > (x1 - x0):
                assert np.all(np.diff(tx * cam.tiles_y + ty) > 0)
                seen["cols"] += 1
            else:
                assert np.all(np.diff(tl.astype(np.int64)) > 0)
                seen["rows"] += 1
        assert seen["rows"] > 100 and (mode != "accutile" or seen["cols"] > 100)


def test_ranges_empty_and_edge_cases():
    assert np.array_equal(oracle.tile_ranges(np.zeros(0, np.uint64), 4), np.zeros((4, 2)))
    keys = (np.array([1, 1, 3], np.uint64) << np.uint64(32))
    r = oracle.tile_ranges(keys, 5)
    assert r.tolist() == [[0, 0], [0, 2], [2, 2], [2, 3], [3, 3]]


# ------------------------------------------------------------ blend

def test_single_gaussian_closed_form():
    cam = scenegen.Camera(64, 48, 64.0, 64.0, 32.0, 24.0, np.eye(3), np.zeros(3))
    sc = single((0.1, -0.05, 2.0), (0.06, 0.03, 0.05), (0.9, 0.1, 0.3, 0.2), 0.8, (0.6, 0.2, -0.4))
    for mode in ("snugbox", "accutile"):
        fr = oracle.render(sc, cam, mode)
        rec = fr.records
        u, v, _, t = rec.geom[0].astype(np.float64)
        a, b, c, sig = rec.conic[0].astype(np.float64)
        ys, xs = np.mgrid[0:cam.height, 0:cam.width] + 0.5
        dx, dy = xs - u, ys - v
        q = a * dx * dx + 2 * b * dx * dy + c * dy * dy
        al = np.minimum(0.99, sig * np.exp(-0.5 * q)) * (q <= t)
        want = al[None] * rec.rgb[0, :3, None, None]
        np.testing.assert_allclose(fr.image, want, atol=2e-6)
        # one contribution exactly where q <= t (away from FP32 rounding of q)
        clear = np.abs(q - t) > 1e-4 * (1.0 + t)
        assert np.array_equal(fr.n_contrib[clear], (q <= t)[clear].astype(np.uint32))


def test_opaque_stack_terminates():
    # Two fully opaque (alpha clamped to 0.99) Gaussians: T = 0.01 after the
    # first and 0.01 * 0.01 < 1e-4 at the second, so only the first is blended.
    cam = scenegen.Camera(32, 32, 32.0, 32.0, 16.0, 16.0, np.eye(3), np.zeros(3))
    sc = scenegen.fixture_scene([(0, 0, 2.0), (0, 0, 2.5), (0, 0, 3.0)], [(0.5,) * 3] * 3,
                                [(1, 0, 0, 0)] * 3, [1.0] * 3,
                                [(1.0, 0, 0), (0, 1.0, 0), (0, 0, 1.0)])
    fr = oracle.render(sc, cam, "accutile")
    c0 = fr.records.rgb[0, :3]
    np.testing.assert_allclose(fr.image[:, 16, 16], F32(0.99) * c0, rtol=1e-6)
    assert fr.n_last[16, 16] == 1
    assert fr.n_contrib[16, 16] == 1
    assert fr.t_final[16, 16] == F32(1.0) - F32(0.99)


def test_two_gaussians_closed_form():
    cam = scenegen.Camera(48, 48, 48.0, 48.0, 24.0, 24.0, np.eye(3), np.zeros(3))
    sc = scenegen.fixture_scene([(0.05, 0, 2.0), (-0.05, 0.02, 3.0)],
                                [(0.08, 0.05, 0.05), (0.1, 0.1, 0.04)],
                                [(1, 0, 0, 0), (0.8, 0, 0.6, 0)], [0.7, 0.9],
                                [(1.0, 0.2, 0.0), (0.1, 0.3, 0.9)])
    fr = oracle.render(sc, cam, "snugbox")
    rec = fr.records
    ys, xs = np.mgrid[0:cam.height, 0:cam.width] + 0.5
    out = np.zeros((3, cam.height, cam.width))
    T = np.ones((cam.height, cam.width))
    n_in = np.zeros((cam.height, cam.width), np.uint32)
    clear = np.ones((cam.height, cam.width), bool)
    for i in (0, 1):  # depth order = index order here
        u, v, _, t = rec.geom[i].astype(np.float64)
        a, b, c, sig = rec.conic[i].astype(np.float64)
        q = a * (xs - u) ** 2 + 2 * b * (xs - u) * (ys - v) + c * (ys - v) ** 2
        al = np.minimum(0.99, sig * np.exp(-0.5 * q)) * (q <= t)
        out += rec.rgb[i, :3, None, None] * (al * T)[None]
        T = T * (1 - al)
        n_in += (q <= t)
        clear &= np.abs(q - t) > 1e-4 * (1.0 + t)
    np.testing.assert_allclose(fr.image, out, atol=3e-6)
    assert np.array_equal(fr.n_contrib[clear], n_in[clear])


@pytest.mark.parametrize("mode", ["snugbox", "accutile"])
def test_tiled_blend_equals_brute_force_c0(mode):
    cam = cam_c0()
    fr = oracle.render(scenegen.scene_c0(), cam, mode)
    ref, amb = oracle.brute_pixels(cam, fr.records, oracle.all_pixels(cam))
    got = fr.image.reshape(3, -1).T.astype(np.float64)
    ok = ~amb & ~fr.ambiguous.reshape(-1)
    assert ok.mean() > 0.995
    assert np.abs(got[ok] - ref[ok]).max() <= 1e-4


def test_3sigma_equals_restricted_brute_force_c0():
    cam = cam_c0()
    fr = oracle.render(scenegen.scene_c0(), cam, "3sigma")
    ref, amb = oracle.brute_pixels(cam, fr.records, oracle.all_pixels(cam), rect_mode="3sigma")
    got = fr.image.reshape(3, -1).T.astype(np.float64)
    ok = ~amb & ~fr.ambiguous.reshape(-1)
    assert np.abs(got[ok] - ref[ok]).max() <= 1e-4


def test_all_three_modes_agree_when_t_le_9():
    # C0 with sigma <= 0.35: every 1/255 support lies inside the 3-sigma square,
    # so the three tile assignments render the same image.
    cam = cam_c0()
    sc = scenegen.scene_c0_lowsigma()
    imgs = {m: oracle.render(sc, cam, m) for m in ("3sigma", "snugbox", "accutile")}
    amb = np.zeros((cam.height, cam.width), bool)
    for f in imgs.values():
        amb |= f.ambiguous
    for m in ("snugbox", "accutile"):
        d = np.abs(imgs[m].image - imgs["3sigma"].image)[:, ~amb]
        assert d.max() <= 1e-6
    assert imgs["accutile"].n_pairs < imgs["snugbox"].n_pairs < imgs["3sigma"].n_pairs

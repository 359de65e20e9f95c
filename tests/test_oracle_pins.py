"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: the paper's
closed forms for an SG lobe (Sec. 3.2 and the Appendix derivation of the colour
compensation), the compositing equation of Sec. 3.1 on configurations with a
closed-form answer, textbook geometry, brute force, and central finite
differences. None of these needs a GPU.
"""
import math

import numpy as np
import pytest

from paper_2509_07021_amd import scenes as S


def _one_gaussian_scene(pos, logscale, quat, op_logit, base, k=0, pmask=None):
    n = len(op_logit)
    z = lambda *shape: np.zeros(shape, np.float64)
    return {
        "pos": np.asarray(pos, np.float64).reshape(3, n),
        "logscale": np.asarray(logscale, np.float64).reshape(3, n),
        "quat": np.asarray(quat, np.float64).reshape(4, n),
        "op_logit": np.asarray(op_logit, np.float64).reshape(n),
        "pmask_logit": None if pmask is None else np.asarray(pmask, np.float64).reshape(n),
        "base": np.asarray(base, np.float64).reshape(3, n),
        "axis": z(k, 3, n) + 1.0, "sharp": z(k, n), "amp": z(k, 3, n), "lmask_logit": None,
    }


# --------------------------------------------------------------- SG colour ----

def test_sg_lobe_value_at_axis_and_antipode(oracle):
    """G(mu) = a and G(-mu) = a e^{-2s} (Eq. for an SG lobe; the two ends of D_i)."""
    rng = np.random.default_rng(11)
    for _ in range(50):
        axis = rng.normal(size=3) * rng.uniform(0.2, 5.0)
        s = rng.uniform(0.3, 60.0)
        a = rng.normal(size=3)
        mu = axis / np.linalg.norm(axis)
        at = oracle.sg_color(np.zeros(3), axis, [s], a, mu)
        anti = oracle.sg_color(np.zeros(3), axis, [s], a, -mu)
        np.testing.assert_allclose(at, a, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(anti, a * math.exp(-2 * s), rtol=1e-12, atol=1e-300)


def test_sg_dynamic_range_matches_importance_formula(oracle):
    """max_v c - min_v c = |a| (1 - e^{-2s}) per channel (Eq. for D_i, Sec. 3.3.2)."""
    rng = np.random.default_rng(12)
    for _ in range(20):
        axis = rng.normal(size=3)
        mu = axis / np.linalg.norm(axis)
        s = rng.uniform(0.5, 40.0)
        a = rng.normal(size=3)
        dirs = rng.normal(size=(2000, 3))
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        dirs = np.vstack([dirs, mu, -mu])
        c = oracle.sg_color_many(np.zeros(3), axis, [s], a, dirs)
        D = c.max(axis=0) - c.min(axis=0)
        np.testing.assert_allclose(D, np.abs(a) * (1 - math.exp(-2 * s)), rtol=1e-12)


def test_sg_zero_sharpness_is_constant(oracle):
    """lambda = 0 makes every lobe direction-independent: c = c0 + sum_k m_k a_k."""
    rng = np.random.default_rng(13)
    k = 4
    base = rng.uniform(size=3)
    axis = rng.normal(size=(k, 3))
    amp = rng.normal(size=(k, 3))
    mask = rng.uniform(size=k)
    dirs = rng.normal(size=(100, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    c = oracle.sg_color_many(base, axis, np.zeros(k), amp, dirs, mask=mask)
    expect = base + (mask[:, None] * amp).sum(0)
    np.testing.assert_allclose(c, np.broadcast_to(expect, c.shape), rtol=1e-14, atol=1e-14)


def test_sg_sphere_mean_matches_compensation_term(oracle):
    """(1/4pi) int_S2 G dv = a (1 - e^{-2s}) / (2s) (Appendix, colour compensation derivation).

    Gauss-Legendre in cos(theta) times the trapezoid rule in phi, in a world frame that
    is NOT aligned with the lobe axis."""
    rng = np.random.default_rng(14)
    nt, nphi = 300, 600
    x, wts = np.polynomial.legendre.leggauss(nt)
    phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    ct = np.repeat(x, nphi)
    st = np.sqrt(1 - ct ** 2)
    ph = np.tile(phi, nt)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1)
    w = np.repeat(wts, nphi) * (2 * np.pi / nphi)
    for s in (0.5, 3.0, 12.0, 45.0):
        axis = rng.normal(size=3)
        a = rng.normal(size=3)
        c = oracle.sg_color_many(np.zeros(3), axis, [s], a, dirs)
        mean = (w[:, None] * c).sum(0) / (4 * np.pi)
        np.testing.assert_allclose(mean, a * (1 - math.exp(-2 * s)) / (2 * s), rtol=1e-9)


def test_paper_parameter_counts(oracle):
    """Colour floats per primitive and rho_s from the paper (golden fixture)."""
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")))
    k = 3
    sc = S.make_scene(10, k, 0, False, False)
    per_lobe = sc.axis.shape[1] + 1 + sc.amp.shape[1]        # axis, sharpness, amplitude
    colour = sc.base.shape[0] + k * per_lobe
    assert per_lobe == g["rho_s"]["value"]
    assert colour == g["colour_floats_3_lobes"]["value"]
    sh3 = g["colour_floats_sh3"]["value"]
    # 3DGS static VRAM: (11 geometric floats + 48 SH floats) x 4 B per Gaussian
    n, mb = g["tt_3dgs"]["gaussians"], g["tt_3dgs"]["static_mb"]
    assert abs(n * (11 + sh3) * 4 / 1e6 - mb) / mb < 0.01


# --------------------------------------------------------------- geometry ----

def _front_cam(w=64, h=64, bg=(0.1, 0.2, 0.05)):
    return S.look_at((0.0, -4.0, 0.0), w, h, bg=bg)


def test_camera_convention_is_exact():
    """The front camera of the tests is an exact axis permutation (so the closed forms are exact)."""
    cam = _front_cam()
    np.testing.assert_array_equal(cam.R, np.array([[1, 0, 0], [0, 0, -1], [0, 1, 0]], np.float32))
    np.testing.assert_array_equal(cam.t, np.array([0, 0, 4], np.float32))
    assert cam.cx == 32 and cam.cy == 32


def test_isotropic_on_axis_footprint(oracle):
    """One isotropic Gaussian on the optical axis: Sigma2 = (f s / z)^2 I + h I, pixel value
    alpha c + (1 - alpha) bg with alpha = min(0.99, o e^{-r^2 / (2 Sigma2)}), background
    outside the disc alpha >= 1/255 (Sec. 3.1 compositing with a single primitive)."""
    cam = _front_cam()
    sigma, logit = 0.2, 2.0
    pl = _one_gaussian_scene([0, 0, 0], [math.log(sigma)] * 3, [1, 0, 0, 0], [logit], [0.3, 0.6, 0.9])
    o = 1 / (1 + math.exp(-logit))
    f = float(cam.fx)
    var = (f * sigma / 4.0) ** 2 + 0.3
    rec = oracle.project(pl, 0, cam, 16)
    assert rec["valid"][0] == 1
    assert rec["u"][0] == 32 and rec["v"][0] == 32 and rec["depth"][0] == 4
    np.testing.assert_allclose(rec["conic"][0], [1 / var, 0, 1 / var], rtol=1e-14, atol=1e-18)
    rho = math.sqrt(2 * math.log(255 * o) * var)
    assert rec["radius"][0] == math.ceil(rho)
    out = oracle.render(pl, 0, [cam], 16)
    img = out["images"][0]
    bg = np.array(cam.bg, np.float64)
    c = np.array([0.3, 0.6, 0.9])
    ys, xs = np.mgrid[0:64, 0:64]
    r2 = (xs + 0.5 - 32) ** 2 + (ys + 0.5 - 32) ** 2
    alpha = np.minimum(0.99, o * np.exp(-0.5 * r2 / var))
    inside = alpha >= 1 / 255
    expect = np.where(inside[None], alpha[None] * c[:, None, None] + (1 - alpha[None]) * bg[:, None, None],
                      bg[:, None, None])
    np.testing.assert_allclose(img, expect, rtol=0, atol=1e-14)
    assert inside.sum() > 50 and (~inside).sum() > 50
    assert np.all(np.sqrt(r2[inside]) <= rho)


@pytest.mark.parametrize("quat,axes", [([1, 0, 0, 0], (0, 2)),
                                        ([math.sqrt(0.5), 0, math.sqrt(0.5), 0], (2, 0))])
def test_anisotropic_rotated_covariance(oracle, quat, axes):
    """Scales (sx, sy, sz) seen along world +y: camera x is world x, camera y is world -z.
    A quarter turn about the view axis swaps which scale lands on which image axis
    (R(q) of a unit quaternion, Sigma = R S S^T R^T, Sigma2 = J W Sigma W^T J^T + h I)."""
    cam = _front_cam()
    sc = np.array([0.3, 0.05, 0.1])
    pl = _one_gaussian_scene([0, 0, 0], np.log(sc), quat, [1.0], [0.5, 0.5, 0.5])
    rec = oracle.project(pl, 0, cam, 16)
    f = float(cam.fx)
    vx = (f * sc[axes[0]] / 4) ** 2 + 0.3
    vy = (f * sc[axes[1]] / 4) ** 2 + 0.3
    np.testing.assert_allclose(rec["conic"][0], [1 / vx, 0, 1 / vy], rtol=1e-12, atol=1e-14)


def test_projection_jacobian_matches_finite_differences(oracle):
    """Sigma2 - h I = s^2 (dp/dmu)(dp/dmu)^T for an isotropic Gaussian, with dp/dmu the
    Jacobian of the projected mean taken by central differences (EWA linearisation)."""
    rng = np.random.default_rng(15)
    cam = S.look_at((0.7, -4.0, 0.9), 96, 64)
    for _ in range(10):
        mu = rng.uniform(-0.8, 0.8, size=3)
        s = 0.07
        pl = _one_gaussian_scene(mu, [math.log(s)] * 3, [1, 0, 0, 0], [1.0], [0.5] * 3)
        rec = oracle.project(pl, 0, cam, 16)
        a, b, c = rec["conic"][0]
        det = a * c - b * b
        S2 = np.array([[c, -b], [-b, a]]) / det
        Jm = np.zeros((2, 3))
        for j in range(3):
            h = 1e-5
            p = mu.copy(); p[j] += h
            m = mu.copy(); m[j] -= h
            rp = oracle.project(_one_gaussian_scene(p, [math.log(s)] * 3, [1, 0, 0, 0], [1.0], [0.5] * 3), 0, cam, 16)
            rm = oracle.project(_one_gaussian_scene(m, [math.log(s)] * 3, [1, 0, 0, 0], [1.0], [0.5] * 3), 0, cam, 16)
            Jm[0, j] = (rp["u"][0] - rm["u"][0]) / (2 * h)
            Jm[1, j] = (rp["v"][0] - rm["v"][0]) / (2 * h)
        expect = s * s * Jm @ Jm.T + 0.3 * np.eye(2)
        np.testing.assert_allclose(S2, expect, rtol=1e-7)


def test_two_gaussian_composite(oracle):
    """C = c1 a1 + c2 a2 (1 - a1) + bg (1 - a1)(1 - a2) for two on-axis Gaussians at
    different depths (Sec. 3.1 compositing); the nearer one is listed second to show the
    order is by depth, not by index."""
    cam = _front_cam()
    s1, s2 = 0.15, 0.3
    pl = _one_gaussian_scene([[0, 0], [1.0, -1.0], [0, 0]],
                             [[math.log(s2), math.log(s1)]] * 3,
                             [[1, 1], [0, 0], [0, 0], [0, 0]], [0.5, 1.5],
                             [[0.9, 0.1], [0.2, 0.8], [0.1, 0.3]])
    out = oracle.render(pl, 0, [cam], 16)
    img = out["images"][0]
    f = float(cam.fx)
    o_near, o_far = 1 / (1 + math.exp(-1.5)), 1 / (1 + math.exp(-0.5))
    var_near = (f * s1 / 3.0) ** 2 + 0.3      # index 1 at y = -1: depth 3
    var_far = (f * s2 / 5.0) ** 2 + 0.3       # index 0 at y = +1: depth 5
    c_near, c_far = np.array([0.1, 0.8, 0.3]), np.array([0.9, 0.2, 0.1])
    bg = np.array(cam.bg)
    checked = 0
    for (x, y) in [(31, 31), (32, 32), (29, 33), (36, 30), (40, 32), (25, 25)]:
        r2 = (x + 0.5 - 32) ** 2 + (y + 0.5 - 32) ** 2
        a1 = min(0.99, o_near * math.exp(-0.5 * r2 / var_near))
        a2 = min(0.99, o_far * math.exp(-0.5 * r2 / var_far))
        if a1 < 1 / 255 or a2 < 1 / 255:
            continue
        expect = c_near * a1 + c_far * a2 * (1 - a1) + bg * (1 - a1) * (1 - a2)
        np.testing.assert_allclose(img[:, y, x], expect, rtol=0, atol=1e-14)
        checked += 1
    assert checked >= 4


def test_empty_scene_is_background(oracle):
    cam = _front_cam(40, 24, bg=(0.25, 0.5, 0.75))
    pl = _one_gaussian_scene(np.zeros((3, 0)), np.zeros((3, 0)), np.zeros((4, 0)), np.zeros(0), np.zeros((3, 0)))
    out = oracle.render(pl, 0, [cam], 8)
    img = out["images"][0]
    np.testing.assert_array_equal(img, np.broadcast_to(np.array(cam.bg)[:, None, None], img.shape))
    assert np.all(out["views"][0]["T"] == 1) and np.all(out["views"][0]["last"] == 0)
    # Gaussians behind the camera or nearer than the near plane contribute nothing either
    pl2 = _one_gaussian_scene([[0, 0.3], [-4.5, -3.9], [0, 0]], [[-2, -2]] * 3, [[1, 1], [0, 0], [0, 0], [0, 0]],
                              [3.0, 3.0], [[1, 1], [1, 1], [1, 1]])
    out2 = oracle.render(pl2, 0, [cam], 8)
    np.testing.assert_array_equal(out2["images"][0], img)
    assert out2["records"]["valid"].sum() == 0


# ---------------------------------------------------------- compositing ----

def test_transmittance_monotone_and_bounded(oracle):
    """T never increases along a pixel's list, and the final T lies in [1e-4, 1]."""
    sc, cams = S.make_workload("small_2k_128px")
    pl = sc.widened()
    out = oracle.render(pl, sc.k, cams, 16)
    T = out["views"][0]["T"]
    assert T.min() >= 1e-4 and T.max() <= 1
    ranges = out["ranges"]
    busiest = np.argsort(ranges[:, 1].astype(np.int64) - ranges[:, 0])[-3:]
    rec = out["records"]
    for t in busiest:
        s, e = int(ranges[t, 0]), int(ranges[t, 1])
        prev = None
        for m in range(0, e - s + 1, max(1, (e - s) // 25)):
            r2 = ranges.copy()
            r2[t, 1] = s + m
            Tm = oracle.blend(cams[0], 16, rec, out["vals"], r2)["T"]
            if prev is not None:
                assert np.all(Tm <= prev)
            prev = Tm


def _planes_tiny(rng, n, k, masks):
    sc = S.random_scene(rng, n, k, masks=masks, spread=0.7, logscale_mu=-2.3)
    return sc.widened(), sc.k


def test_tiled_equals_bruteforce_and_tile_invariance(oracle):
    rng = np.random.default_rng(21)
    for trial in range(12):
        n = int(rng.integers(0, 60))
        k = int(rng.integers(0, 5))
        pl, k = _planes_tiny(rng, n, k, masks=bool(trial % 2))
        eye = rng.normal(size=3)
        eye = 3.0 * eye / np.linalg.norm(eye)
        cam = S.look_at(eye, int(rng.integers(17, 70)), int(rng.integers(17, 70)),
                        bg=tuple(rng.uniform(size=3)))
        ref = None
        for tile in (8, 16, 32):
            out = oracle.render(pl, k, [cam], tile)
            img = out["images"][0]
            rec = out["records"]
            bf = oracle.bruteforce(cam, rec, rec["valid"])
            np.testing.assert_allclose(img, bf["image"], rtol=0, atol=1e-12)
            np.testing.assert_array_equal(out["views"][0]["T"], bf["T"])
            if ref is None:
                ref = img
            else:
                np.testing.assert_array_equal(img, ref)


def test_key_table_structure(oracle):
    """Keys ascend; ranges partition [0, P); every listed (tile, record) pair lies inside the
    record's rectangle; and -- the property the compositor relies on -- every pixel where a
    record's alpha reaches 1/255 (brute force over the pixels, in numpy) lies in a tile listed for
    that record. Tile culling inside the rectangle must drop pairs."""
    sc, cams = S.make_workload("small_2k_128px")
    cams = cams + [S.look_at((3.0, 1.0, 2.0), 72, 40)]
    pl = sc.widened()
    tile = 16
    out = oracle.render(pl, sc.k, cams, tile)
    keys, vals, ranges, off = out["keys"], out["vals"], out["ranges"], out["tile_off"]
    order = np.lexsort((vals, keys))
    np.testing.assert_array_equal(order, np.arange(len(keys)))
    nz = ranges[:, 1] > ranges[:, 0]
    cover = np.zeros(len(keys), np.int32)
    for t in np.nonzero(nz)[0]:
        s, e = ranges[t]
        cover[s:e] += 1
        assert np.all((keys[s:e] >> np.uint64(32)) == t)
    assert np.all(cover == 1)
    got = set(zip((keys >> np.uint64(32)).astype(np.int64).tolist(), vals.astype(np.int64).tolist()))
    rec = out["records"]
    n = sc.n
    rect_total = 0
    for g in np.nonzero(rec["valid"])[0]:
        vi = g // n
        cam = cams[vi]
        tx = (cam.width + tile - 1) // tile
        u, v, r = rec["u"][g], rec["v"][g], rec["radius"][g]
        xl, xh, yl, yh = math.floor(u) - r, math.floor(u) + r, math.floor(v) - r, math.floor(v) + r
        if xh < 0 or yh < 0 or xl > cam.width - 1 or yl > cam.height - 1:
            continue
        xl, yl = max(xl, 0), max(yl, 0)
        xh, yh = min(xh, cam.width - 1), min(yh, cam.height - 1)
        rect = {(int(off[vi]) + ty * tx + tx_) for ty in range(yl // tile, yh // tile + 1)
                for tx_ in range(xl // tile, xh // tile + 1)}
        rect_total += len(rect)
        listed = {t for t in rect if (t, int(g)) in got}
        # pixels of the whole image where this record passes the compositor's alpha test
        ys, xs = np.mgrid[0:cam.height, 0:cam.width]
        dx, dy = xs + 0.5 - u, ys + 0.5 - v
        a, b, c = rec["conic"][g]
        q = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy
        alpha = np.minimum(0.99, rec["o"][g] * np.exp(q))
        hit = (alpha >= 1 / 255) & (q <= 0)
        need = {int(off[vi]) + (int(y) // tile) * tx + int(x) // tile for y, x in zip(*np.nonzero(hit))}
        assert need <= listed, (g, need - listed)
    assert len(got) < rect_total
    assert all(k[1] < n * len(cams) for k in got)
    dep = rec["depth"].astype(np.float32).view(np.uint32)
    np.testing.assert_array_equal((keys & np.uint64(0xFFFFFFFF)).astype(np.uint32), dep[vals])


def _qp_box_min(C, m, box):
    """min over the box of (p - m)' C (p - m) by scipy's bound-constrained quasi-Newton solver (a library
    routine that knows nothing of edges or vertices), from several starting points."""
    from scipy.optimize import minimize
    f = lambda p: float((p - m) @ C @ (p - m))
    jac = lambda p: 2.0 * C @ (p - m)
    lo, hi = np.array([box[0], box[2]]), np.array([box[1], box[3]])
    best = np.inf
    for x0 in (np.clip(m, lo, hi), (lo + hi) / 2, lo, hi, np.array([lo[0], hi[1]]), np.array([hi[0], lo[1]])):
        r = minimize(f, x0, jac=jac, method="L-BFGS-B", bounds=list(zip(lo, hi)),
                     options={"ftol": 1e-15, "gtol": 1e-13, "maxiter": 500})
        best = min(best, float(r.fun))
    return best


def _random_conic(rng, cond_max=1e4):
    """A positive definite 2 x 2 conic with a random orientation and condition number up to cond_max."""
    lam1 = 10 ** rng.uniform(-3, 1)
    lam2 = lam1 * 10 ** rng.uniform(0, np.log10(cond_max))
    th = rng.uniform(0, np.pi)
    Rm = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    return Rm @ np.diag([lam1, lam2]) @ Rm.T


def test_box_minimum_against_library_qp(oracle):
    """The oracle's tile predicate rests on the minimum of the footprint's quadratic form over a box. It
    equals the bound-constrained minimum found by a library solver, for means inside, beside and
    diagonal to the box, conics up to condition 1e4, and boxes down to a single pixel centre; and no point
    of a dense grid over the box goes below it."""
    rng = np.random.default_rng(17)
    us, vs, cs, bs, ref = [], [], [], [], []
    for trial in range(300):
        C = _random_conic(rng)
        x0, y0 = rng.uniform(-20, 20, 2)
        wbox, hbox = (0.0, 0.0) if trial % 10 == 0 else rng.uniform(0, 16, 2)
        box = np.array([x0, x0 + wbox, y0, y0 + hbox])
        m = np.array([x0, y0]) + rng.uniform(-25, 40, 2)
        if trial % 10 == 3:  # mean inside the box
            m = np.array([x0 + rng.uniform(0, 1) * wbox, y0 + rng.uniform(0, 1) * hbox])
        us.append(m[0]); vs.append(m[1]); cs.append([C[0, 0], C[0, 1], C[1, 1]]); bs.append(box)
        ref.append(_qp_box_min(C, m, box))
    got = oracle.box_min(np.array(us), np.array(vs), np.array(cs), np.array(bs))
    ref = np.array(ref)
    np.testing.assert_allclose(got, ref, rtol=1e-7, atol=1e-9)
    assert (got == 0).sum() >= 5 and (got > 0).sum() >= 200  # both the inside and the boundary cases
    for i in range(0, 300, 7):
        gx = np.linspace(bs[i][0], bs[i][1], 161)
        gy = np.linspace(bs[i][2], bs[i][3], 161)
        X, Y = np.meshgrid(gx - us[i], gy - vs[i])
        a, b, c = cs[i]
        grid = a * X * X + 2 * b * X * Y + c * Y * Y
        assert grid.min() >= got[i] * (1 - 1e-12) - 1e-12
    # a conic that is not positive definite bounds nothing
    assert oracle.box_min([0.0], [0.0], [[1.0, 2.0, 1.0]], [[5, 6, 5, 6]])[0] == -np.inf


def test_key_table_is_exactly_the_reached_tiles(oracle):
    """Both directions of the tile predicate, at every tile of every rectangle, on needle-shaped and round
    footprints and images whose edges cut tiles: a tile is listed exactly when the footprint ellipse at the
    record's level k reaches the tile's pixel-centre box, with the box minimum taken by a library solver
    (pairs whose solver minimum lies within 1e-7 k of k are left out as undecidable by it). A listing that
    is too wide or too narrow, a wrong box edge or a wrong level fails here."""
    rng = np.random.default_rng(23)
    sc = S.random_scene(rng, 120, 1, masks=True, spread=0.8, logscale_mu=-3.0)
    sc.logscale[0, :40] = rng.uniform(-0.8, 0.0, 40).astype(sc.logscale.dtype)
    sc.logscale[1:, :40] = rng.uniform(-6.5, -5.0, (2, 40)).astype(sc.logscale.dtype)
    pl = sc.widened()
    cams = [S.look_at((0, -3.5, 0.4), 100, 72), S.look_at((2.5, -2.0, 1.0), 56, 50)]
    checked = listed_n = skipped = 0
    for tile in (8, 16):
        out = oracle.render(pl, sc.k, cams, tile)
        rec, keys, vals, off = out["records"], out["keys"], out["vals"], out["tile_off"]
        got = set(zip((keys >> np.uint64(32)).astype(np.int64).tolist(), vals.astype(np.int64).tolist()))
        for g in np.nonzero(rec["valid"])[0]:
            vi = g // sc.n
            cam = cams[vi]
            tx_n = (cam.width + tile - 1) // tile
            u, v, r = rec["u"][g], rec["v"][g], rec["radius"][g]
            a, b, c = rec["conic"][g]
            C = np.array([[a, b], [b, c]])
            k = rec["cutoff"][g]
            xl, xh = max(math.floor(u) - r, 0), min(math.floor(u) + r, cam.width - 1)
            yl, yh = max(math.floor(v) - r, 0), min(math.floor(v) + r, cam.height - 1)
            if xl > xh or yl > yh:
                continue
            for ty in range(yl // tile, yh // tile + 1):
                for tx in range(xl // tile, xh // tile + 1):
                    box = (tx * tile + 0.5, min((tx + 1) * tile, cam.width) - 0.5,
                           ty * tile + 0.5, min((ty + 1) * tile, cam.height) - 0.5)
                    qmin = _qp_box_min(C, np.array([u, v]), box)
                    if abs(qmin - k) <= 1e-7 * k:
                        skipped += 1
                        continue
                    listed = (int(off[vi]) + ty * tx_n + tx, int(g)) in got
                    assert listed == (qmin <= k), (tile, g, tx, ty, qmin, k, listed)
                    checked += 1
                    listed_n += listed
    assert checked > 2000 and checked - listed_n > 300 and skipped <= 2, (checked, listed_n, skipped)
    # the level bounds the alpha >= 1/255 support (alpha = o e^{-Q/2}) and exceeds it by a small margin only
    v = rec["valid"].astype(bool)
    k0 = 2.0 * np.log(255.0 * rec["o"][v])
    assert np.all(rec["cutoff"][v] >= k0) and np.all(rec["cutoff"][v] <= 1.005 * k0 + 2e-4)


# -------------------------------------------------------------- gradients ----

def _fd_check(oracle, pl, k, cams, tile, weights, rng, per_plane=10):
    grads, _ = oracle.render_backward(pl, k, cams, tile, weights)
    checked = 0
    for p in oracle.PLANES:
        if pl.get(p) is None or pl[p].size == 0:
            continue
        flat = pl[p].reshape(-1)
        idx = rng.choice(flat.size, size=min(flat.size, per_plane), replace=False)
        fd, ok = oracle.fd_gradient(pl, k, cams, tile, weights, p, idx, rel_h=1e-6)
        an = grads[p].reshape(-1)[idx]
        scale = np.abs(grads[p]).max()
        tol = 1e-4 * np.maximum(np.abs(an), 1e-3 * scale) + 1e-8
        bad = ok & (np.abs(fd - an) > tol)
        assert not bad.any(), (p, idx[bad], fd[bad], an[bad])
        checked += int(ok.sum())
    return checked


def test_gradients_match_central_differences(oracle):
    """Analytic FP64 gradient of L = sum(w * image) vs central differences, every raw
    parameter class, two views, soft masks on."""
    rng = np.random.default_rng(31)
    sc = S.random_scene(rng, 30, 3, masks=True, spread=0.6, logscale_mu=-2.0)
    cams = [S.look_at((0, -3, 0.5), 48, 40, bg=(0.2, 0.1, 0.3)), S.look_at((2.5, -1.5, 1.0), 40, 32)]
    w = S.loss_weights(cams, 9)
    assert _fd_check(oracle, sc.widened(), sc.k, cams, 8, w, rng) > 80


def test_gradients_match_central_differences_clamped_jacobian(oracle):
    """Gaussians near the image border and beyond the 1.3x field-of-view clamp."""
    rng = np.random.default_rng(32)
    sc = S.random_scene(rng, 25, 2, masks=False, spread=2.5, logscale_mu=-1.2)
    cams = [S.look_at((0, -2.2, 0.0), 40, 40)]
    w = S.loss_weights(cams, 10)
    assert _fd_check(oracle, sc.widened(), sc.k, cams, 16, w, rng) > 60


def test_masked_crop_gradients_match_central_differences(oracle):
    """The masked 1M workload's 500-Gaussian crop (the 500 Gaussians nearest the first view's axis,
    its centred 64x64 window, soft masks on): the analytic FP64 gradient against central
    differences for a sample of coordinates of every parameter plane, mask logits included. The
    same crop is the GPU's masked-gradient parity case."""
    scene, cams = S.make_workload("masked_1m_1080p", n=200_000)
    crop = scene.subset(S.axis_nearest(scene, cams[0], 500))
    cam = S.crop_camera(cams[0], 64, 64)
    w = S.loss_weights([cam], 3)
    rng = np.random.default_rng(33)
    assert _fd_check(oracle, crop.widened(), crop.k, [cam], 16, w, rng, per_plane=16) >= 140


def test_blend_backward_recursion_equals_direct_sum(oracle):
    """dL/dalpha by the back-to-front background recursion equals the O(n^2) term-by-term
    derivative of C = sum c_i a_i T_i + T_final bg."""
    sc, cams = S.make_workload("small_2k_128px")
    cams = [S.look_at((0.0, -4.0, 0.0), 64, 64, bg=(0.3, 0.2, 0.1))]
    pl = sc.widened()
    out = oracle.render(pl, sc.k, cams, 16)
    w = S.loss_weights(cams, 3)
    g_rec = oracle.blend_backward(cams[0], 16, out["records"], out["vals"], out["ranges"], w[0])
    g_dir = oracle.blend_backward(cams[0], 16, out["records"], out["vals"], out["ranges"], w[0], direct=True)
    np.testing.assert_allclose(g_rec, g_dir, rtol=1e-9, atol=1e-12 * np.abs(g_dir).max())


def test_saturated_masks_reproduce_mask_free_path(oracle):
    """sigmoid(+40) == 1 in FP64, so saturated masks give exactly the mask-free image and gradient."""
    rng = np.random.default_rng(41)
    sc = S.random_scene(rng, 40, 3, masks=False, spread=0.7, logscale_mu=-2.3)
    pl = sc.widened()
    cams = [S.look_at((0.3, -3.0, 0.4), 40, 40)]
    w = S.loss_weights(cams, 5)
    a = oracle.render(pl, sc.k, cams, 8)
    pm = dict(pl)
    pm["pmask_logit"] = np.full(sc.n, 40.0)
    pm["lmask_logit"] = np.full((sc.k, sc.n), 40.0)
    b = oracle.render(pm, sc.k, cams, 8)
    np.testing.assert_array_equal(a["images"][0], b["images"][0])
    ga, _ = oracle.render_backward(pl, sc.k, cams, 8, w)
    gb, _ = oracle.render_backward(pm, sc.k, cams, 8, w)
    for p in ("pos", "logscale", "quat", "op_logit", "base", "axis", "sharp", "amp"):
        np.testing.assert_array_equal(ga[p], gb[p])

"""Pins of the oracle's pruning definitions (Sec. 3.3, Alg. 1 and the Appendix's proximal
operators) against closed forms, invariants, brute force and a toy problem whose answer is known."""
import math

import numpy as np

from paper_2509_07021_amd import scenes as S

from test_oracle_pins import _front_cam, _one_gaussian_scene


def test_importance_single_gaussian_is_sum_of_alpha(oracle):
    """One Gaussian: T = 1 in front of it, so I = sum over pixels of alpha (closed form)."""
    cam = _front_cam()
    sigma, logit = 0.2, 1.5
    pl = _one_gaussian_scene([0, 0, 0], [math.log(sigma)] * 3, [1, 0, 0, 0], [logit], [0.3, 0.6, 0.9])
    o = 1 / (1 + math.exp(-logit))
    var = (float(cam.fx) * sigma / 4.0) ** 2 + 0.3
    ys, xs = np.mgrid[0:64, 0:64]
    r2 = (xs + 0.5 - 32) ** 2 + (ys + 0.5 - 32) ** 2
    alpha = np.minimum(0.99, o * np.exp(-0.5 * r2 / var))
    expect = alpha[alpha >= 1 / 255].sum()
    got = oracle.importance(pl, 0, [cam], 16)
    np.testing.assert_allclose(got, [expect], rtol=1e-13)


def test_importance_sums_to_opacity_of_each_pixel(oracle):
    """sum_i alpha_i T_i = 1 - T_final per pixel (the product telescopes), so the importance
    scores of one view sum to sum_p (1 - T_final(p))."""
    rng = np.random.default_rng(4)
    sc = S.random_scene(rng, 300, 2, masks=True, spread=0.8, logscale_mu=-2.5)
    cams = [S.look_at((0.4, -3.0, 0.6), 64, 48), S.look_at((2.0, 2.0, 1.0), 40, 56)]
    pl = sc.widened()
    fwd = oracle.render(pl, sc.k, cams, 8)
    imp = oracle.importance(pl, sc.k, cams, 8)
    expect = sum((1.0 - v["T"]).sum() for v in fwd["views"])
    np.testing.assert_allclose(imp.sum(), expect, rtol=1e-12)
    assert np.all(imp >= 0)


def test_topk_keep_brute_force_and_ties():
    rng = np.random.default_rng(5)
    for _ in range(30):
        n = int(rng.integers(0, 40))
        score = rng.integers(0, 6, size=n).astype(np.float64)  # many ties
        kappa = int(rng.integers(-2, n + 3))
        from oracle import oracle as O
        keep = O.topk_keep(score, kappa)
        ranked = sorted(range(n), key=lambda i: (-score[i], i))[:max(0, min(kappa, n))]
        assert set(np.nonzero(keep)[0].tolist()) == set(ranked)


def test_lobe_dynamic_range_matches_the_sg_model(oracle):
    """D = |a| (1 - e^{-2z}) equals the Euclidean norm of the per-channel max - min of the lobe
    over the sphere (Eq. for D_i), evaluated with the oracle's SG colour."""
    rng = np.random.default_rng(6)
    k, n = 3, 5
    z = rng.uniform(0.2, 30.0, size=(k, n))
    amp = rng.normal(size=(k, 3, n))
    D = oracle.lobe_dynamic_range(z, amp)
    for l in range(k):
        for i in range(n):
            axis = rng.normal(size=3)
            mu = axis / np.linalg.norm(axis)
            dirs = np.vstack([mu, -mu, rng.normal(size=(500, 3))])
            dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
            c = oracle.sg_color_many(np.zeros(3), axis, [z[l, i]], amp[l, :, i], dirs)
            rng_ch = c.max(0) - c.min(0)
            np.testing.assert_allclose(np.linalg.norm(rng_ch), D[l, i], rtol=1e-12)


def test_prox_keeps_the_budget(oracle):
    rng = np.random.default_rng(7)
    n, k = 200, 3
    o, lam_o, imp = rng.uniform(size=n), rng.normal(0, 0.1, n), rng.uniform(size=n)
    s, lam_s, amp = rng.uniform(0.5, 20, (k, n)), rng.normal(0, 0.5, (k, n)), rng.normal(size=(k, 3, n))
    o_t, s_t = oracle.prox(o, lam_o, imp, 50, s, lam_s, amp, 120)
    assert np.count_nonzero(o_t) <= 50 and np.count_nonzero(s_t) <= 120
    kept = o_t != 0
    np.testing.assert_array_equal(o_t[kept], (o + lam_o)[kept])
    assert imp[kept].min() >= imp[~kept].max()
    D = oracle.lobe_dynamic_range(s + lam_s, amp)
    ks = s_t != 0
    np.testing.assert_array_equal(s_t[ks], (s + lam_s)[ks])
    assert D[ks].min() >= D[~ks].max()


def _admm_step(oracle, x, xt, lam, c, kappa, eta, delta):
    grad = oracle.penalty_grad(x - c, delta, x, xt, lam)
    x = x - eta * grad
    z = x + lam
    xt = np.where(oracle.topk_keep(np.abs(z), kappa), z, 0.0)
    lam = oracle.dual_update(lam, x, xt)
    return x, xt, lam


def test_admm_fixed_point_of_a_sparse_least_squares_toy(oracle):
    """Alg. 1's gradient, proximal and dual steps on L(x) = |x - c|^2 / 2 with |x|_0 <= kappa
    (magnitude-based selection). By hand from the three update equations, a fixed point is
    x = x_tilde = c on the kappa largest |c| and 0 elsewhere, lambda = 0 on that support and
    c / delta off it (kept when delta > max_off |c| / min_on |c|). One step must leave it
    unchanged, and small perturbations must decay -- a sign error in the penalty term or the
    dual update breaks both."""
    rng = np.random.default_rng(8)
    n, kappa = 40, 7
    c = rng.normal(size=n)
    sup = oracle.topk_keep(np.abs(c), kappa)
    eta, delta = 0.1, 2.0
    x_star = np.where(sup, c, 0.0)
    lam_star = np.where(sup, 0.0, c / delta)
    x, xt, lam = _admm_step(oracle, x_star, x_star, lam_star, c, kappa, eta, delta)
    np.testing.assert_allclose(x, x_star, atol=1e-15)
    np.testing.assert_allclose(xt, x_star, atol=1e-15)
    np.testing.assert_allclose(lam, lam_star, atol=1e-15)
    pert = 1e-3 * rng.normal(size=(3, n))
    x, xt, lam = x_star + pert[0], x_star + pert[1] * sup, lam_star + pert[2]
    d0 = np.abs(x - x_star).max() + np.abs(lam - lam_star).max()
    for _ in range(300):
        x, xt, lam = _admm_step(oracle, x, xt, lam, c, kappa, eta, delta)
    d1 = np.abs(x - x_star).max() + np.abs(lam - lam_star).max()
    assert d1 < 1e-6 * d0
    np.testing.assert_array_equal(xt != 0, sup)

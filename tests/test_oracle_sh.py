"""Pins of the oracle's spherical-harmonic colour (the 3DGS colour model that the paper's SG colour
replaces, Sec. 1 and Sec. 3.2; used for the same-renderer comparison): orthonormality over the
sphere, the addition theorem degree by degree, derivatives by finite differences, the offset and
clamp on a one-Gaussian scene, and end-to-end gradients by central differences."""
import math

import numpy as np

from paper_2509_07021_amd import scenes as S

from test_oracle_pins import _front_cam, _one_gaussian_scene


def _sphere_grid(nt=64, nphi=128):
    x, wts = np.polynomial.legendre.leggauss(nt)
    phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    ct = np.repeat(x, nphi)
    st = np.sqrt(1 - ct ** 2)
    ph = np.tile(phi, nt)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1)
    return dirs, np.repeat(wts, nphi) * (2 * np.pi / nphi)


def test_basis_is_orthonormal(oracle):
    dirs, w = _sphere_grid()
    Y, _ = oracle.sh_basis(dirs)
    gram = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-12)


def test_addition_theorem_per_degree(oracle):
    """sum_m Y_lm(a) Y_lm(b) = (2l + 1) / (4 pi) P_l(a . b) for each degree l <= 3 (independent of
    the sign convention, it fixes every polynomial up to a rotation of its degree's subspace)."""
    rng = np.random.default_rng(90)
    a = rng.normal(size=(200, 3)); a /= np.linalg.norm(a, axis=1, keepdims=True)
    b = rng.normal(size=(200, 3)); b /= np.linalg.norm(b, axis=1, keepdims=True)
    Ya, _ = oracle.sh_basis(a)
    Yb, _ = oracle.sh_basis(b)
    t = (a * b).sum(1)
    P = [np.ones_like(t), t, 0.5 * (3 * t ** 2 - 1), 0.5 * (5 * t ** 3 - 3 * t)]
    for l in range(4):
        sl = slice(l * l, (l + 1) ** 2)
        np.testing.assert_allclose((Ya[:, sl] * Yb[:, sl]).sum(1), (2 * l + 1) / (4 * math.pi) * P[l], atol=1e-13)


def test_basis_derivatives_match_finite_differences(oracle):
    rng = np.random.default_rng(91)
    d = rng.normal(size=(50, 3))
    _, dY = oracle.sh_basis(d)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3); e[a] = h
        Yp, _ = oracle.sh_basis(d + e)
        Ym, _ = oracle.sh_basis(d - e)
        np.testing.assert_allclose(dY[:, :, a], (Yp - Ym) / (2 * h), rtol=1e-7, atol=1e-8)


def test_dc_colour_offset_and_clamp(oracle):
    """Only DC coefficients: colour = max(0, sh0 / (2 sqrt(pi)) + 1/2) in every direction."""
    cam = _front_cam()
    pl = _one_gaussian_scene([0, 0, 0], [math.log(0.2)] * 3, [1, 0, 0, 0], [2.0], [0.0, 0.0, 0.0])
    pl["base"] = None
    sh = np.zeros((16, 3, 1))
    sh[0, :, 0] = [0.7, -0.4, -3.0]
    pl["sh"] = sh
    rec = oracle.project(pl, 0, cam, 16)
    expect = np.maximum(0.0, sh[0, :, 0] / (2 * math.sqrt(math.pi)) + 0.5)
    np.testing.assert_allclose(rec["rgb"][0], expect, rtol=1e-15)
    assert expect[2] == 0.0


def test_sh_render_gradients_match_central_differences(oracle):
    rng = np.random.default_rng(92)
    sc = S.sh_scene(S.random_scene(rng, 25, 0, masks=True, spread=0.6, logscale_mu=-2.0), 92)
    cams = [S.look_at((0, -3, 0.5), 40, 40, bg=(0.2, 0.1, 0.3)), S.look_at((2.0, -2.0, 1.0), 32, 32)]
    w = S.loss_weights(cams, 14)
    pl = sc.widened()
    assert pl["sh"].shape == (16, 3, 25)
    grads, _ = oracle.render_backward(pl, 0, cams, 8, w)
    checked = 0
    for p in ("sh", "pos", "logscale", "op_logit"):
        idx = rng.choice(pl[p].size, size=10, replace=False)
        fd, ok = oracle.fd_gradient(pl, 0, cams, 8, w, p, idx, rel_h=1e-6)
        an = grads[p].reshape(-1)[idx]
        tol = 1e-4 * np.maximum(np.abs(an), 1e-3 * np.abs(grads[p]).max()) + 1e-8
        assert not (ok & (np.abs(fd - an) > tol)).any(), (p, fd, an)
        checked += int(ok.sum())
    assert checked >= 30

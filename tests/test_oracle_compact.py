"""Pins of the oracle's post-processing (Sec. 3.3, post-processing procedure; the compensation
equation and its derivation in the Appendix) and of its compressed-row (ragged lobe) renderer,
against quadrature over the sphere, brute-force enumeration, the renderer's own culling rule and
the dense renderer (which the finite-difference pins cover)."""
import math

import numpy as np
import pytest

from paper_2509_07021_amd import scenes as S


def _sphere_grid(nt=200, nphi=400):
    x, wts = np.polynomial.legendre.leggauss(nt)
    phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    ct = np.repeat(x, nphi)
    st = np.sqrt(1 - ct ** 2)
    ph = np.tile(phi, nt)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1)
    w = np.repeat(wts, nphi) * (2 * np.pi / nphi) / (4 * np.pi)  # weights of the sphere average
    return dirs, w


def test_sphere_mean_factor_against_quadrature(oracle):
    """The compensation factor is the average of e^{s (mu . d - 1)} over the sphere, for any s
    (the derivation's integral holds for s of either sign; s = 0 is the limit 1)."""
    dirs, w = _sphere_grid()
    rng = np.random.default_rng(60)
    for s in (-0.7, 0.0, 1e-3, 0.4, 0.999, 2.5, 9.0):
        axis = rng.normal(size=3)
        c = oracle.sg_color_many(np.zeros(3), axis, [s], np.ones(3), dirs)[:, 0]
        np.testing.assert_allclose(oracle.sphere_mean_factor([s])[0], (w * c).sum(), rtol=1e-10)


def _lobe_list(pl, k, i):
    """(sharpness, axis, amplitude, mask) of Gaussian i's lobes in slot order, by plain indexing."""
    out = []
    n = len(pl["op_logit"])
    if pl.get("lobe_off") is None:
        for l in range(k):
            m = 1.0 if pl["lmask_logit"] is None else 1 / (1 + math.exp(-pl["lmask_logit"][l, i]))
            out.append((pl["sharp"][l, i], pl["axis"][l, :, i], pl["amp"][l, :, i], m, l * n + i))
    else:
        for j in range(pl["lobe_off"][i], pl["lobe_off"][i + 1]):
            m = 1.0 if pl["lmask_logit"] is None else 1 / (1 + math.exp(-pl["lmask_logit"][j]))
            out.append((pl["sharp"][j], pl["axis"][:, j], pl["amp"][:, j], m, j))
    return out


@pytest.mark.parametrize("ragged,masks", [(False, True), (False, False), (True, True), (True, False)])
def test_compaction_by_enumeration(oracle, ragged, masks):
    """Kept Gaussians, kept lobes, their order, offsets, index maps, compensated base colours
    and folded masks, written out Gaussian by Gaussian in plain Python."""
    rng = np.random.default_rng(61 + 2 * ragged + masks)
    sc = (S.ragged_scene(rng, 70, 3, masks) if ragged else S.random_scene(rng, 70, 3, masks))
    pl = sc.widened()
    pl["sharp"] = pl["sharp"] * rng.choice([0.01, 1.0], size=pl["sharp"].shape)  # about half below 1
    tau_o, tau_s = 0.4, 1.0
    out = oracle.compact(pl, sc.k, tau_o, tau_s)
    kept, offs, lsrc = [], [0], []
    for i in range(sc.n):
        o = 1 / (1 + math.exp(-pl["op_logit"][i]))
        if masks:
            o *= 1 / (1 + math.exp(-pl["pmask_logit"][i]))
        if not o >= tau_o:
            continue
        kept.append(i)
        base = pl["base"][:, i].copy()
        j0 = offs[-1]
        for s, ax, a, m, src in _lobe_list(pl, sc.k, i):
            if s >= tau_s:
                lsrc.append(src)
                jj = len(lsrc) - 1
                np.testing.assert_array_equal(out["axis"][:, jj], ax)
                assert out["sharp"][jj] == s
                np.testing.assert_allclose(out["amp"][:, jj], m * a, rtol=1e-15)
            else:
                base += m * a * (1 - math.exp(-2 * s)) / (2 * s)
        offs.append(len(lsrc))
        jk = len(kept) - 1
        np.testing.assert_allclose(out["base"][:, jk], base, rtol=1e-14, atol=1e-15)
        np.testing.assert_allclose(1 / (1 + np.exp(-out["op_logit"][jk])), o, rtol=1e-13)
        for p in ("pos", "logscale", "quat"):
            np.testing.assert_array_equal(out[p][:, jk], pl[p][:, i])
        assert offs[-1] - j0 <= sc.k
    np.testing.assert_array_equal(out["kept"], kept)
    np.testing.assert_array_equal(out["lobe_off"], offs)
    np.testing.assert_array_equal(out["lobe_src"], lsrc)
    assert 0 < len(kept) < sc.n and 0 < len(lsrc)


def test_compensation_keeps_the_sphere_average_colour(oracle):
    """Dropping lobes with compensation leaves each Gaussian's colour averaged over all view
    directions unchanged (what the compensation equation minimises the loss of), checked by
    quadrature of the SG colour before and after."""
    rng = np.random.default_rng(62)
    sc = S.random_scene(rng, 12, 4, masks=True)
    pl = sc.widened()
    pl["op_logit"] = np.full(sc.n, 3.0)
    out = oracle.compact(pl, sc.k, 0.0, 20.0)       # drops every lobe with s < 20
    assert len(out["kept"]) == sc.n and len(out["lobe_src"]) < sc.n * sc.k
    dirs, w = _sphere_grid(120, 240)
    for i in range(sc.n):
        lobes = _lobe_list(pl, sc.k, i)
        c0 = oracle.sg_color_many(pl["base"][:, i], np.array([l[1] for l in lobes]), [l[0] for l in lobes],
                                  np.array([l[2] for l in lobes]), dirs, mask=[l[3] for l in lobes])
        a, b = out["lobe_off"][i], out["lobe_off"][i + 1]
        if b > a:
            c1 = oracle.sg_color_many(out["base"][:, i], out["axis"][:, a:b].T, out["sharp"][a:b],
                                      out["amp"][:, a:b].T, dirs)
        else:
            c1 = np.broadcast_to(out["base"][:, i], c0.shape)
        np.testing.assert_allclose((w[:, None] * c1).sum(0), (w[:, None] * c0).sum(0), rtol=1e-9, atol=1e-12)


def test_removing_culled_gaussians_changes_no_pixel(oracle):
    """With the opacity threshold at the renderer's own 1/255 cut and no lobe dropped, the
    compacted (compressed-row, masks folded) scene renders the same images."""
    rng = np.random.default_rng(63)
    sc = S.random_scene(rng, 150, 3, masks=True, spread=0.8, logscale_mu=-2.4)
    pl = sc.widened()
    pl["op_logit"] = pl["op_logit"] - rng.choice([0.0, 7.0], size=sc.n)  # a third or so below 1/255
    cams = [S.look_at((0.3, -3.0, 0.6), 64, 48, bg=(0.1, 0.2, 0.3)), S.look_at((2.0, 2.0, 1.5), 40, 56)]
    out = oracle.compact(pl, sc.k, 1 / 255, -np.inf)
    assert 0 < len(out["kept"]) < sc.n and len(out["lobe_src"]) == sc.k * len(out["kept"])
    a = oracle.render(pl, sc.k, cams, 16)
    b = oracle.render(out, sc.k, cams, 16)
    for ia, ib in zip(a["images"], b["images"]):
        np.testing.assert_allclose(ib, ia, rtol=0, atol=1e-12)


def _pad_dense(pl, kmax):
    """Dense planes holding a compressed-row scene: each Gaussian's lobes in its first slots,
    the rest zero-amplitude lobes (they add exactly nothing)."""
    n = len(pl["op_logit"])
    off = pl["lobe_off"]
    d = {p: pl[p] for p in ("pos", "logscale", "quat", "op_logit", "pmask_logit", "base")}
    d["axis"] = np.zeros((kmax, 3, n)); d["axis"][:, 0, :] = 1.0
    d["sharp"] = np.ones((kmax, n))
    d["amp"] = np.zeros((kmax, 3, n))
    d["lmask_logit"] = None if pl["lmask_logit"] is None else np.zeros((kmax, n))
    where = []
    for i in range(n):
        for l, j in enumerate(range(off[i], off[i + 1])):
            d["axis"][l, :, i] = pl["axis"][:, j]
            d["sharp"][l, i] = pl["sharp"][j]
            d["amp"][l, :, i] = pl["amp"][:, j]
            if pl["lmask_logit"] is not None:
                d["lmask_logit"][l, i] = pl["lmask_logit"][j]
            where.append((j, l, i))
    return d, where


def test_ragged_renderer_equals_padded_dense_renderer(oracle):
    """The compressed-row renderer and its gradient equal the dense ones on the same lobes."""
    rng = np.random.default_rng(64)
    sc = S.ragged_scene(rng, 60, 3, masks=True, spread=0.7, logscale_mu=-2.3)
    pl = sc.widened()
    dense, where = _pad_dense(pl, sc.k)
    cams = [S.look_at((0.2, -3.0, 0.5), 48, 40), S.look_at((-2.0, 2.2, 1.0), 40, 40, bg=(0.3, 0.3, 0.3))]
    w = S.loss_weights(cams, 12)
    a = oracle.render(pl, sc.k, cams, 8)
    b = oracle.render(dense, sc.k, cams, 8)
    for ia, ib in zip(a["images"], b["images"]):
        np.testing.assert_array_equal(ia, ib)
    ga, _ = oracle.render_backward(pl, sc.k, cams, 8, w, fwd=a)
    gb, _ = oracle.render_backward(dense, sc.k, cams, 8, w, fwd=b)
    for p in ("pos", "logscale", "quat", "op_logit", "pmask_logit", "base"):
        np.testing.assert_array_equal(ga[p], gb[p])
    for j, l, i in where:
        np.testing.assert_array_equal(ga["axis"][:, j], gb["axis"][l, :, i])
        assert ga["sharp"][j] == gb["sharp"][l, i] and ga["lmask_logit"][j] == gb["lmask_logit"][l, i]
        np.testing.assert_array_equal(ga["amp"][:, j], gb["amp"][l, :, i])


def test_ragged_gradients_match_central_differences(oracle):
    rng = np.random.default_rng(65)
    sc = S.ragged_scene(rng, 25, 3, masks=True, spread=0.6, logscale_mu=-2.0)
    cams = [S.look_at((0, -3, 0.5), 40, 40, bg=(0.2, 0.1, 0.3))]
    w = S.loss_weights(cams, 13)
    pl = sc.widened()
    grads, _ = oracle.render_backward(pl, sc.k, cams, 8, w)
    for p in ("axis", "sharp", "amp", "lmask_logit"):
        idx = rng.choice(pl[p].size, size=8, replace=False)
        fd, ok = oracle.fd_gradient(pl, sc.k, cams, 8, w, p, idx, rel_h=1e-6)
        an = grads[p].reshape(-1)[idx]
        tol = 1e-4 * np.maximum(np.abs(an), 1e-3 * np.abs(grads[p]).max()) + 1e-8
        assert ok.sum() >= 6 and not (ok & (np.abs(fd - an) > tol)).any(), (p, fd, an)


def test_malformed_offsets_cull_the_gaussian(oracle):
    rng = np.random.default_rng(66)
    sc = S.ragged_scene(rng, 8, 2, masks=False)
    pl = sc.widened()
    pl["lobe_off"] = pl["lobe_off"].copy()
    cam = S.look_at((0, -3, 0), 32, 32)
    pl["lobe_off"][3] = pl["lobe_off"][4] + 1  # Gaussian 3 has a negative count, 2 one too many
    rec = oracle.project(pl, sc.k, cam, 16)
    assert rec["valid"][3] == 0

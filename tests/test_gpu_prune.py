"""GPU parity of the pruning steps (importance score, lobe dynamic range, top-kappa selection,
proximal, dual and penalty updates) against the oracle's plain definitions."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_07021_amd import render as R
from paper_2509_07021_amd import scenes as S

from gpu_util import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2509_07021_amd import prune as PR  # noqa: E402


def test_select_topk_is_exact_with_ties():
    rng = np.random.default_rng(1)
    for n in (1, 2, 17, 1000, 65537, 1 << 20):
        for ties in (False, True):
            score = (rng.integers(0, 50, size=n) if ties else rng.normal(size=n)).astype(np.float32)
            if n > 10:
                score[: n // 10] = -score[: n // 10]
                score[5] = -0.0
                score[6] = 0.0
            for kappa in sorted({0, 1, n // 3, n - 1, n, n + 5}):
                log(f"topk n={n} ties={ties} kappa={kappa}")
                keep = PR.select_topk(torch.from_numpy(score).cuda(), kappa).cpu().numpy().astype(bool)
                np.testing.assert_array_equal(keep, O.topk_keep(score.astype(np.float64), kappa))


def test_lobe_range_matches_oracle():
    rng = np.random.default_rng(2)
    k, n = 4, 10000
    s = rng.uniform(-1, 50, size=(k, n)).astype(np.float32)
    lam = rng.normal(0, 0.5, size=(k, n)).astype(np.float32)
    amp = rng.normal(0, 0.2, size=(k, 3, n)).astype(np.float32)
    D = PR.lobe_range(torch.from_numpy(s).cuda(), torch.from_numpy(amp).cuda(), torch.from_numpy(lam).cuda())
    z = s.astype(np.float32) + lam.astype(np.float32)  # the sum the kernel forms in FP32
    ref = O.lobe_dynamic_range(z.astype(np.float64), amp.astype(np.float64))
    np.testing.assert_allclose(D.cpu().numpy(), ref, rtol=2e-6, atol=1e-7)


def test_prox_dual_penalty_match_definitions():
    rng = np.random.default_rng(3)
    n = 50000
    x, lam, g = (rng.normal(size=n).astype(np.float32) for _ in range(3))
    keep = (rng.random(n) < 0.3).astype(np.uint8)
    tx, tl, tg, tk = (torch.from_numpy(a).cuda() for a in (x, lam, g, keep))
    xt = PR.prox_apply(tx, tl, tk)
    ref_xt = np.where(keep.astype(bool), x + lam, np.float32(0))
    np.testing.assert_array_equal(xt.cpu().numpy(), ref_xt)
    lam2 = PR.dual_update_(tl.clone(), tx, xt)
    np.testing.assert_array_equal(lam2.cpu().numpy(), lam + (x - ref_xt))
    g2 = PR.penalty_grad_(tg.clone(), 0.0005 * 11, tx, xt, tl)
    ref = O.penalty_grad(g, 0.0005 * 11, x, ref_xt, lam)
    np.testing.assert_allclose(g2.cpu().numpy(), ref, rtol=1e-6, atol=1e-7)


def _decision_slack(fwd, cams, tile, n, band=2e-4):
    """Per Gaussian, the most its importance can move through decisions near a threshold.

    At a pixel the oracle flags, a decision within `band` (relative: the oracle's flag band) of the
    alpha threshold 1/255 or of the termination threshold 1e-4 may go either way on the GPU. The
    pixel's list is walked front to back with the oracle's exact transmittance beside an interval
    [T_lo, T_hi] holding every transmittance the GPU can reach through such decisions (T_lo = 0
    once it may have stopped); each entry's GPU weight then lies in [alpha T_lo, alpha T_hi] (or
    may be 0 where it may be excluded), and its distance from the oracle's weight is the entry's
    slack. Before the first such decision both sides agree (slack 0). Alpha's clamp at 0.99 is
    continuous and moves no weight."""
    rec = fwd["records"]
    slack = np.zeros(n, np.float64)
    a_min, t_min = 1.0 / 255.0, 1e-4
    for vi, cam in enumerate(cams):
        ys, xs = np.nonzero(fwd["views"][vi]["flag"])
        tiles_x = (cam.width + tile - 1) // tile
        rv = fwd["ranges"][fwd["tile_off"][vi]:fwd["tile_off"][vi + 1]]
        for y, x in zip(ys, xs):
            s, e = rv[(y // tile) * tiles_x + x // tile]
            g = fwd["vals"][s:e].astype(np.int64)
            dx, dy = x + 0.5 - rec["u"][g], y + 0.5 - rec["v"][g]
            a, b, c = rec["conic"][g].T
            power = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy
            alpha = np.where(power <= 0, np.minimum(0.99, rec["o"][g] * np.exp(np.minimum(power, 0.0))), 0.0)
            T_o, o_alive, T_lo, T_hi = 1.0, True, 1.0, 1.0
            for gi, al in zip(g, alpha):
                if not o_alive and T_hi == 0.0:
                    break
                w_o = 0.0
                if o_alive and al >= a_min:
                    if T_o * (1.0 - al) < t_min:
                        o_alive = False
                    else:
                        w_o = al * T_o
                        T_o *= 1.0 - al
                maybe_in = abs(al - a_min) <= band * a_min
                sure_in = al > a_min * (1.0 + band)
                if T_hi == 0.0 or not (maybe_in or sure_in):
                    lo_w = hi_w = 0.0
                else:
                    n_lo, n_hi = T_lo * (1.0 - al), T_hi * (1.0 - al)
                    stops = n_hi < t_min * (1.0 - band)
                    goes_on = n_lo > t_min * (1.0 + band)
                    lo_w = al * T_lo if (sure_in and goes_on) else 0.0
                    hi_w = 0.0 if stops else al * T_hi
                    T_lo = n_lo if goes_on else 0.0
                    T_hi = 0.0 if stops else (T_hi if maybe_in else n_hi)
                d = max(abs(w_o - lo_w), abs(w_o - hi_w))
                if d > 1e-12 * max(w_o, 1e-30):
                    slack[gi % n] += d * (1.0 + 1e-6)
    return slack


def test_importance_and_prox_step_on_the_masked_workload():
    """Importance over 3 views of a 20k subsample of the masked 1M workload against the oracle,
    element by element: within 1e-4 relative (FP32 accumulation of the weights alpha * T) plus,
    for the Gaussians behind a decision near a threshold at some pixel, the most another decision
    there can move their score (_decision_slack). Then the whole
    factorised proximal step: the selections are bit-exact given the GPU's scores."""
    scene, cams = S.make_workload("masked_1m_1080p", n=200_000)
    idx = np.sort(np.random.default_rng(103).choice(scene.n, 20_000, replace=False))
    sub = scene.subset(idx)
    cams = [S.crop_camera(c, 480, 270) for c in S.ring_cameras(3, 3)]
    ds = R.DeviceScene.from_scene(sub)
    ref = O.importance(sub.widened(), sub.k, cams, 16)
    slack = _decision_slack(O.render(sub.widened(), sub.k, cams, 16), cams, 16, sub.n)
    loose = slack > 1e-3 * ref
    log(f"importance: {int((slack > 0).sum())} of {sub.n} Gaussians behind a decision near a threshold, "
        f"{int(loose.sum())} with slack above 1e-3 of their score")
    assert loose.mean() < 0.01
    scores = []
    for cfg in (R.Config(16, 64), R.Config(16, 64, subtile=8)):   # both blend instances
        imp = PR.importance(ds, cams, cfg)[1].cpu().numpy().astype(np.float64)
        scores.append(imp)
        err = np.abs(imp - ref)
        bound = 1e-4 * ref + 1e-7 + slack
        log(f"importance subtile={cfg.subtile}: total {imp.sum():.4f} vs {ref.sum():.4f}, "
            f"worst err / bound {float((err / bound).max()):.3f}, "
            f"unflagged worst rel {float((err / (ref + 1e-7))[slack == 0].max()):.2e}")
        assert (err <= bound).all(), np.argmax(err / bound)
        np.testing.assert_allclose(imp.sum(), ref.sum(), rtol=1e-5)
    imp = scores[0]
    # the proximal step, kappa_o = 40% of the primitives and kappa_s = 50% of the lobes
    rng = np.random.default_rng(9)
    o = torch.sigmoid(ds.planes["op_logit"]).contiguous()
    lam_o = torch.from_numpy(rng.normal(0, 0.01, sub.n).astype(np.float32)).cuda()
    lam_s = torch.from_numpy(rng.normal(0, 0.1, (sub.k, sub.n)).astype(np.float32)).cuda()
    imp_t = torch.from_numpy(imp.astype(np.float32)).cuda()
    o_t, s_t = PR.prox_step(o, lam_o, imp_t, int(0.4 * sub.n), ds.planes["sharp"], lam_s, ds.planes["amp"],
                            int(0.5 * sub.n * sub.k))
    D = PR.lobe_range(ds.planes["sharp"], ds.planes["amp"], lam_s).cpu().numpy().astype(np.float64)
    keep_o = O.topk_keep(imp.astype(np.float32).astype(np.float64), int(0.4 * sub.n))
    keep_s = O.topk_keep(D.ravel(), int(0.5 * sub.n * sub.k)).reshape(D.shape)
    zo = (o + lam_o).cpu().numpy()
    zs = (ds.planes["sharp"] + lam_s).cpu().numpy()
    np.testing.assert_array_equal(o_t.cpu().numpy(), np.where(keep_o, zo, 0))
    np.testing.assert_array_equal(s_t.cpu().numpy(), np.where(keep_s, zs, 0))

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


def test_importance_and_prox_step_on_the_masked_workload():
    """Importance over 3 views of a 20k subsample of the masked 1M workload against the oracle,
    then the whole factorised proximal step: the selections are bit-exact given the GPU's scores."""
    scene, cams = S.make_workload("masked_1m_1080p", n=200_000)
    idx = np.sort(np.random.default_rng(103).choice(scene.n, 20_000, replace=False))
    sub = scene.subset(idx)
    cams = [S.crop_camera(c, 480, 270) for c in S.ring_cameras(3, 3)]
    ds = R.DeviceScene.from_scene(sub)
    _, imp = PR.importance(ds, cams, R.Config(16, 64))
    imp = imp.cpu().numpy().astype(np.float64)
    ref = O.importance(sub.widened(), sub.k, cams, 16)
    log(f"importance: total {imp.sum():.4f} vs {ref.sum():.4f}")
    np.testing.assert_allclose(imp.sum(), ref.sum(), rtol=1e-5)
    close = np.abs(imp - ref) <= 1e-4 * np.maximum(ref, 1.0)
    assert close.mean() > 0.995 and np.abs(imp - ref).max() < 0.05
    # the sub-tile blend's importance instance gives the same scores
    _, imp8 = PR.importance(ds, cams, R.Config(16, 64, subtile=8))
    imp8 = imp8.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(imp8.sum(), ref.sum(), rtol=1e-5)
    assert (np.abs(imp8 - ref) <= 1e-4 * np.maximum(ref, 1.0)).mean() > 0.995
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

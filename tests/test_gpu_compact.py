"""GPU parity of the post-processing (Sec. 3.3: threshold pruning of Gaussians and lobes, colour
compensation, compaction into the compressed-row lobe layout) and of the renderer on
compressed-row scenes, against the FP64 oracle. Index maps, offsets and bit-copied planes are
compared exactly; computed values (folded opacity logit, compensated base colour, mask-scaled
amplitude) to one unit in the last place of their storage dtype."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_07021_amd import _lib as L
from paper_2509_07021_amd import prune as P
from paper_2509_07021_amd import render as R
from paper_2509_07021_amd import scenes as S

from gpu_util import IMG_TOL, grad_close, gpu_run, log, scene_from_device

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

ULP = {"f32": 2.0 ** -23, "f16": 2.0 ** -10, "bf16": 2.0 ** -7}
TINY = {"f32": 1e-37, "f16": 6e-8, "bf16": 1e-37}


def _opacity(pl):
    o = 1 / (1 + np.exp(-pl["op_logit"]))
    if pl.get("pmask_logit") is not None:
        o = o * (1 / (1 + np.exp(-pl["pmask_logit"])))
    return o


def _compare_compaction(scene, tau_o, tau_s):
    log(f"compaction n={scene.n} k={scene.k} ragged={scene.ragged} dt={scene.dt_geom}/{scene.dt_color}/"
        f"{scene.dt_amp} thresholds {tau_o} {tau_s}")
    pl = scene.widened()
    o = _opacity(pl)
    if o.size and np.isfinite(tau_o) and tau_o > 0:
        # FP64 on both sides; keep every decision clear of the last-place differences of exp
        assert np.min(np.abs(o - tau_o)) > 1e-9 * tau_o
    ds = R.DeviceScene.from_scene(scene)
    cds, kept, lsrc = P.compact(ds, tau_o, tau_s)
    torch.cuda.synchronize()
    ref = O.compact(pl, scene.k, tau_o, tau_s)
    np.testing.assert_array_equal(kept.cpu().numpy(), ref["kept"])
    np.testing.assert_array_equal(cds.lobe_off.cpu().numpy(), ref["lobe_off"])
    np.testing.assert_array_equal(lsrc.cpu().numpy(), ref["lobe_src"])
    assert cds.n == len(ref["kept"]) and cds.n_lobes == len(ref["lobe_src"]) and cds.k == scene.k
    got_scene = scene_from_device(cds)
    got = got_scene.widened()
    for p in ("pos", "logscale", "quat", "axis", "sharp"):
        np.testing.assert_array_equal(got[p], ref[p].reshape(got[p].shape), err_msg=p)
    for p, dt in (("op_logit", scene.dt_geom), ("base", scene.dt_color), ("amp", scene.dt_amp)):
        r = ref[p].reshape(got[p].shape)
        bound = ULP[dt] * np.abs(r) + TINY[dt]
        d = np.abs(got[p] - r)
        assert np.all(d <= bound), (p, float((d / bound).max()))
    assert got["pmask_logit"] is None and got["lmask_logit"] is None
    return cds, got_scene, ref


def _post_admm_small(n, seed, masks=True, k=3):
    return S.post_admm(S.make_scene(n, k, seed, clustered=False, masks=masks), seed)


def test_compaction_dense_masked():
    _compare_compaction(_post_admm_small(20_000, 71), 0.01, 1.0)


def test_compaction_dense_without_masks():
    _compare_compaction(_post_admm_small(20_000, 72, masks=False), 0.05, 1.0)


def test_compaction_ragged_input():
    rng = np.random.default_rng(73)
    sc = S.ragged_scene(rng, 15_000, 4, masks=True)
    sc.sharp[rng.random(sc.sharp.shape) < 0.5] *= 0.02
    _compare_compaction(sc, 0.3, 1.0)


def test_compaction_reduced_precision():
    sc = _post_admm_small(20_000, 74).stored("f16", "f16", "bf16")
    _compare_compaction(sc, 0.01, 1.0)


def test_compaction_edge_cases():
    sc = _post_admm_small(3_000, 75)
    cds, _, _ = _compare_compaction(sc, 2.0, 1.0)          # nothing passes an opacity above 1
    assert cds.n == 0 and cds.n_lobes == 0
    cds, _, _ = _compare_compaction(sc, 0.0, -np.inf)      # everything kept, no lobe dropped
    assert cds.n == sc.n and cds.n_lobes == sc.n * sc.k
    cds, _, _ = _compare_compaction(sc, 0.0, np.inf)       # every lobe folded into the base
    assert cds.n == sc.n and cds.n_lobes == 0
    _compare_compaction(sc.subset(np.zeros(0, np.int64)), 0.01, 1.0)   # empty scene
    _compare_compaction(S.make_scene(2_000, 0, 76, clustered=False, masks=True), 0.1, 1.0)   # k = 0


def test_compaction_rejects_malformed_offsets():
    rng = np.random.default_rng(77)
    sc = S.ragged_scene(rng, 500, 3, masks=False)
    sc.lobe_off = sc.lobe_off.copy()
    sc.lobe_off[100] = sc.lobe_off[101] + 2   # a negative count: the kernels' offset check rejects it
    ds = R.DeviceScene.from_scene(sc)
    with pytest.raises(L.MegsError) as e:
        P.compact(ds, 0.01, 1.0)
    assert e.value.status == L.MEGS_ERR_ARG and "lobe_off" in str(e.value)
    with pytest.raises(L.MegsError) as e:
        R.forward(ds, [S.look_at((0, -3, 0), 64, 64)], R.Config(16, 64))
    assert e.value.status == L.MEGS_ERR_ARG


def _oracle_weights(scene, cams, tile, seed):
    fwd = O.render(scene.widened(), scene.k, cams, tile)
    w = S.loss_weights(cams, seed)
    return fwd, [wi * (1 - vw["flag"])[None].astype(np.float32) for wi, vw in zip(w, fwd["views"])]


def _render_parity(scene, cams, cfg, seed=8):
    """End-to-end images and raw-parameter gradients of a compressed-row scene."""
    log(f"ragged render n={scene.n} lobes={scene.n_lobes} k={scene.k} views={len(cams)} tile={cfg.tile}")
    fwd, w = _oracle_weights(scene, cams, cfg.tile, seed)
    g = gpu_run(scene, cams, cfg, weights=w)
    for vi in range(len(cams)):
        ok = fwd["views"][vi]["flag"] == 0
        d = np.abs(g["images"][vi] - fwd["images"][vi])[:, ok]
        assert d.max() <= IMG_TOL, (vi, d.max())
    gr, _ = O.render_backward(scene.widened(), scene.k, cams, cfg.tile, w, fwd=fwd)
    for p in O.PLANES:
        if gr[p] is not None:
            assert g["grads"][p].shape == gr[p].shape, p
            grad_close(p, g["grads"][p], gr[p])
    return g


def test_ragged_random_scene_renders_and_differentiates():
    rng = np.random.default_rng(78)
    sc = S.ragged_scene(rng, 3000, 3, masks=True, spread=1.0, logscale_mu=-3.0)
    cams = [S.look_at((0.3, -3.5, 0.6), 160, 120, bg=(0.1, 0.2, 0.3)), S.look_at((2.5, 2.0, 1.2), 96, 136)]
    for tile, waves in ((16, 4), (8, 1)):
        _render_parity(sc, cams, R.Config(tile, 64, waves=waves))


def test_compacted_scene_renders_and_differentiates():
    """The GPU's own compaction output, rendered on the GPU, against the oracle on those planes."""
    sc = S.post_admm(S.make_scene(30_000, 3, 79, clustered=True, masks=True), 79)
    cds, host, _ = _compare_compaction(sc, 0.01, 1.0)
    cams = [S.look_at((0.5, -6.0, 1.0), 192, 108)]
    _render_parity(host, cams, R.Config(16, 64))


def test_ragged_reduced_precision_and_no_lobes():
    rng = np.random.default_rng(80)
    sc = S.ragged_scene(rng, 2000, 3, masks=False, logscale_mu=-2.8).stored("f16", "f16", "bf16")
    cams = [S.look_at((0.0, -3.2, 0.4), 128, 96)]
    _render_parity(sc, cams, R.Config(16, 64))
    none = S.ragged_scene(rng, 1500, 3, masks=True, logscale_mu=-2.8)
    none = none.subset(np.arange(none.n))
    none.lobe_off = np.zeros(none.n + 1, np.int32)
    for p in ("axis", "sharp", "amp", "lmask_logit"):
        a = getattr(none, p)
        setattr(none, p, np.ascontiguousarray(a[..., :0]))
    _render_parity(none, cams, R.Config(16, 64))

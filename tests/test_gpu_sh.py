"""GPU parity of the spherical-harmonic colour variant (3DGS's colour model, run through the same
renderer for the bytes-per-Gaussian comparison with SG colour), against the FP64 oracle: images
and every raw gradient, degrees 0-3, with masks and in FP16 storage."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_07021_amd import render as R
from paper_2509_07021_amd import scenes as S

from gpu_util import IMG_TOL, grad_close, gpu_run, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)


def _parity(scene, cams, cfg, seed=15):
    log(f"sh render n={scene.n} planes={scene.sh.shape} dt={scene.dt_color} views={len(cams)} tile={cfg.tile}")
    fwd = O.render(scene.widened(), 0, cams, cfg.tile)
    w = [wi * (1 - vw["flag"])[None].astype(np.float32) for wi, vw in zip(S.loss_weights(cams, seed), fwd["views"])]
    g = gpu_run(scene, cams, cfg, weights=w)
    for vi in range(len(cams)):
        ok = fwd["views"][vi]["flag"] == 0
        d = np.abs(g["images"][vi] - fwd["images"][vi])[:, ok]
        assert d.max() <= IMG_TOL, (vi, d.max())
    gr, _ = O.render_backward(scene.widened(), 0, cams, cfg.tile, w, fwd=fwd)
    checked = 0
    for p in O.PLANES:
        if gr[p] is not None:
            grad_close(p, g["grads"][p], gr[p])
            checked += 1
    assert gr["sh"] is not None and checked >= 5


@pytest.mark.parametrize("degree", [0, 1, 2, 3])
def test_sh_degrees(degree):
    rng = np.random.default_rng(110 + degree)
    sc = S.sh_scene(S.random_scene(rng, 2500, 0, masks=True, spread=1.0, logscale_mu=-3.0), 110 + degree, degree)
    cams = [S.look_at((0.3, -3.5, 0.6), 160, 120, bg=(0.1, 0.2, 0.3)), S.look_at((2.5, 2.0, 1.2), 96, 136)]
    _parity(sc, cams, R.Config(16, 64))


def test_sh_fp16_storage_and_clamp():
    rng = np.random.default_rng(115)
    sc = S.sh_scene(S.random_scene(rng, 2500, 0, masks=False, spread=1.0, logscale_mu=-3.0), 115, 3)
    sc.sh[0] -= 1.5          # push part of the colours below zero: the clamp and its zero gradient
    sc = sc.stored("f16", "f16", "f32")
    cams = [S.look_at((0.0, -3.2, 0.4), 128, 96)]
    _parity(sc, cams, R.Config(8, 64, waves=1))

"""GPU tests of the differentiable entry point: render() through RenderFn, the torch.autograd.Function
wrapping the forward and the back-to-front replay backward, then loss.backward().

The gradients that reach the leaf planes' .grad are compared with the FP64 oracle's gradient and with the
library's backward called directly, and their dtype must be the plane's storage dtype (autograd casts the
library's FP32 gradients for FP16 and BF16 planes)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_07021_amd import render as R
from paper_2509_07021_amd import scenes as S

from gpu_util import grad_close, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)


def _masked_weights(scene, cams, tile, seed):
    fwd = O.render(scene.widened(), scene.k, cams, tile)
    w = S.loss_weights(cams, seed)
    return fwd, [wi * (1 - vw["flag"])[None].astype(np.float32) for wi, vw in zip(w, fwd["views"])]


def _autograd_grads(scene, cams, cfg, weights):
    """render() on leaf planes with requires_grad, L = sum w * image, L.backward(); returns the .grad
    tensors and the images."""
    ds = R.DeviceScene.from_scene(scene)
    for t in ds.planes.values():
        if t is not None:
            t.requires_grad_(True)
    imgs = R.render(ds, cams, cfg)
    loss = sum((torch.from_numpy(w).cuda() * img).sum() for w, img in zip(weights, imgs))
    loss.backward()
    torch.cuda.synchronize()
    return ds, imgs, {p: t.grad for p, t in ds.planes.items() if t is not None}


@pytest.mark.parametrize("cfg", [R.Config(32, 64, subtile=8), R.Config(16, 64)], ids=["sub8", "tile16"])
def test_render_autograd_fp32(cfg):
    """FP32 planes: .grad after loss.backward() equals the oracle's gradient (the 1e-4 tolerances) and
    the library's backward called directly; images equal the oracle's."""
    scene, cams = S.make_workload("small_2k_128px")
    cams = cams + [S.look_at((2.0, -3.0, 1.5), 100, 60, bg=(0.2, 0.2, 0.2))]
    log(f"autograd fp32 {cfg}")
    fwd, w = _masked_weights(scene, cams, cfg.tile, 13)
    ds, imgs, grads = _autograd_grads(scene, cams, cfg, w)
    for vi, img in enumerate(imgs):
        ok = fwd["views"][vi]["flag"] == 0
        d = np.abs(img.detach().cpu().numpy() - fwd["images"][vi])[:, ok]
        assert d.max() <= 1e-5, (vi, d.max())
    ref, _ = O.render_backward(scene.widened(), scene.k, cams, cfg.tile, w, fwd=fwd)
    plain = {p: t.detach() for p, t in ds.planes.items() if t is not None}
    fr = R.forward(ds, cams, cfg, planes=plain)
    direct = R.backward(ds, fr, torch.from_numpy(np.concatenate([x.reshape(-1) for x in w])).cuda(), planes=plain)
    for p, g in grads.items():
        assert g is not None and g.dtype == torch.float32 and g.shape == ds.planes[p].shape, p
        gh = g.cpu().numpy().astype(np.float64)
        grad_close(p, gh, ref[p])
        grad_close(f"direct {p}", gh, direct[p].cpu().numpy().astype(np.float64), rel=1e-5)


@pytest.mark.parametrize("amp_dt", ["f16", "bf16"])
def test_render_autograd_reduced_precision(amp_dt):
    """FP16 planes (amplitudes in FP16 or BF16): .grad has each plane's dtype and equals the FP32
    gradient of the library's backward rounded to that dtype (within one unit in its last place: the
    FP32 sums' order differs between two runs), which in turn meets the oracle's gradient of the
    stored values at the 1e-4 tolerances."""
    full, cams = S.make_workload("clustered_200k_720p", n=20_000)
    scene = full.stored("f16", "f16", amp_dt)
    cams = [S.crop_camera(cams[0], 320, 180)]
    cfg = R.Config(32, 64, subtile=8)
    log(f"autograd f16/{amp_dt}")
    fwd, w = _masked_weights(scene, cams, cfg.tile, 17)
    ds, imgs, grads = _autograd_grads(scene, cams, cfg, w)
    ref, _ = O.render_backward(scene.widened(), scene.k, cams, cfg.tile, w, fwd=fwd)
    plain = {p: t.detach() for p, t in ds.planes.items() if t is not None}
    fr = R.forward(ds, cams, cfg, planes=plain)
    direct = R.backward(ds, fr, torch.from_numpy(np.concatenate([x.reshape(-1) for x in w])).cuda(), planes=plain)
    for p, g in grads.items():
        t = ds.planes[p]
        assert g is not None and g.dtype == t.dtype and g.shape == t.shape, (p, g.dtype, t.dtype)
        g32 = direct[p]
        grad_close(f"direct {p}", g32.cpu().numpy().astype(np.float64), ref[p])
        # one unit in the last place of the storage dtype at the FP32 value, plus a floor for values
        # the FP32 sums put on either side of a rounding boundary near zero
        eps = {torch.float16: 2.0 ** -10, torch.bfloat16: 2.0 ** -7}[t.dtype]
        tiny = {torch.float16: 2.0 ** -24, torch.bfloat16: 1e-38}[t.dtype]
        bound = eps * g32.abs() + tiny + 1e-5 * g32.abs().max()
        err = (g.float() - g32).abs()
        assert bool((err <= bound).all()), (p, float((err / bound).max()))

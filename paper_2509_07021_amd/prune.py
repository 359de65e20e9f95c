"""PyTorch-facing wrappers of the memory-constrained optimisation steps (Sec. 3.3, Alg. 1; the
Appendix's proximal operators). The work runs in libmegs.so's kernels; tensors are contiguous
FP32 CUDA tensors (uint8 for selection masks)."""
from __future__ import annotations

import ctypes
from typing import Sequence

import torch

from . import _lib as L
from . import render as R


def _p(t):
    return None if t is None else t.data_ptr()


def _s():
    return torch.cuda.current_stream().cuda_stream


def importance(dscene: R.DeviceScene, cams: Sequence, cfg: R.Config = R.Config(), out: torch.Tensor = None):
    """Renders the views and returns (flat images, importance [n]): every Gaussian's blending
    weights alpha * T summed over all pixels of all views (added into `out` when given)."""
    lib = L.load()
    npix = sum(c.width * c.height for c in cams)
    images = torch.empty(3 * npix, dtype=torch.float32, device="cuda")
    imp = out if out is not None else torch.zeros(dscene.n, dtype=torch.float32, device="cuda")
    alloc = R.TorchAllocator()
    st = L.MegsState()
    sc = dscene.struct()
    c = cfg.struct()
    L.check(lib.megs_render_importance(ctypes.byref(sc), R.cameras_struct(cams), len(cams), ctypes.byref(c),
                                       alloc.fn, None, images.data_ptr(), imp.data_ptr(), ctypes.byref(st), _s()))
    return images, imp


def lobe_range(sharp: torch.Tensor, amp: torch.Tensor, lam: torch.Tensor = None) -> torch.Tensor:
    """D = |a| (1 - exp(-2 (sharp + lam))) per lobe; sharp [k][n], amp [k][3][n]."""
    k, n = sharp.shape
    D = torch.empty_like(sharp)
    L.check(L.load().megs_lobe_range(n, k, _p(sharp), _p(lam), _p(amp), _p(D), _s()))
    return D


def select_topk(score: torch.Tensor, kappa: int) -> torch.Tensor:
    """uint8 mask of the kappa largest scores (ties to the lower index)."""
    score = score.contiguous().view(-1)
    keep = torch.empty(score.numel(), dtype=torch.uint8, device=score.device)
    alloc = R.TorchAllocator()
    L.check(L.load().megs_select_topk(_p(score), score.numel(), int(kappa), alloc.fn, None, _p(keep), _s()))
    keep._alloc_keepalive = alloc
    return keep


def prox_apply(x: torch.Tensor, lam: torch.Tensor, keep: torch.Tensor) -> torch.Tensor:
    xt = torch.empty_like(x)
    L.check(L.load().megs_prox_apply(x.numel(), _p(x), _p(lam), _p(keep), _p(xt), _s()))
    return xt


def dual_update_(lam: torch.Tensor, x: torch.Tensor, x_tilde: torch.Tensor) -> torch.Tensor:
    L.check(L.load().megs_dual_update(lam.numel(), _p(lam), _p(x), _p(x_tilde), _s()))
    return lam


def penalty_grad_(grad: torch.Tensor, delta: float, x: torch.Tensor, x_tilde: torch.Tensor,
                  lam: torch.Tensor) -> torch.Tensor:
    L.check(L.load().megs_penalty_grad(grad.numel(), float(delta), _p(x), _p(x_tilde), _p(lam), _p(grad), _s()))
    return grad


def prox_step(o, lam_o, imp, kappa_o, sharp, lam_s, amp, kappa_s):
    """Factorised proximal step of Alg. 1: o_tilde keeps the kappa_o entries of o + lambda_o with
    the highest importance; s_tilde keeps the kappa_s lobes of s + lambda_s with the highest
    dynamic range D (at s + lambda_s)."""
    o_t = prox_apply(o, lam_o, select_topk(imp, kappa_o))
    D = lobe_range(sharp, amp, lam_s)
    s_t = prox_apply(sharp, lam_s, select_topk(D, kappa_s).view(sharp.shape))
    return o_t, s_t


def compact(dscene: R.DeviceScene, opacity_min: float, sharp_min: float = 1.0):
    """Post-processing (Sec. 3.3): drops Gaussians with opacity below opacity_min and lobes with
    sharpness below sharp_min (the paper's lobe threshold is 1), folding each dropped lobe's
    average over all directions into the base colour and the soft masks into opacity and amplitude.

    Returns (compacted DeviceScene in the compressed-row layout, kept int32 [n'], lobe_src
    int32 [n_lobes']): the source Gaussian of each kept Gaussian and the source sharpness element
    of each kept lobe. Synchronises the stream once (the output sizes are data-dependent)."""
    lib = L.load()
    alloc = R.TorchAllocator()
    out = L.MegsCompacted()
    sc = dscene.struct()
    L.check(lib.megs_compact(ctypes.byref(sc), float(opacity_min), float(sharp_min), alloc.fn, None, _s(),
                             ctypes.byref(out)))
    r = out.scene
    n, nl = int(r.n), int(r.n_lobes)
    dg, dc, da = (R._TORCH_DT[d] for d in dscene.dt)

    def view(ptr, shape, dtype):
        count = 1
        for s in shape:
            count *= s
        if count == 0:
            return torch.empty(shape, dtype=dtype, device="cuda")
        return alloc.view(ptr, count, dtype).view(shape)

    planes = {
        "pos": view(r.pos, (3, n), dg), "logscale": view(r.logscale, (3, n), dg),
        "quat": view(r.quat, (4, n), dg), "op_logit": view(r.op_logit, (n,), dg), "pmask_logit": None,
        "base": view(r.base, (3, n), dc), "axis": view(r.axis, (3, nl), dc), "sharp": view(r.sharp, (nl,), dc),
        "amp": view(r.amp, (3, nl), da), "lmask_logit": None,
    }
    lobe_off = alloc.view(r.lobe_off, n + 1, torch.int32)
    kept = view(out.kept, (n,), torch.int32)
    lobe_src = view(out.lobe_src, (nl,), torch.int32)
    ds = R.DeviceScene(planes, int(r.k), *dscene.dt, lobe_off=lobe_off, n_lobes=nl, keepalive=alloc)
    return ds, kept, lobe_src

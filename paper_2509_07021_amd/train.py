"""Training-step pieces around the renderer: the 3DGS photometric loss (L1 + D-SSIM) with its
gradient and Adam on parameter planes stored in FP32, FP16 or BF16 (the paper trains with 3DGS's
loss, hyperparameters and optimiser; Appendix, experimental details). The work runs in
libmegs.so's kernels."""
from __future__ import annotations

import ctypes
from typing import Dict, Optional, Sequence

import torch

from . import _lib as L
from . import render as R

# 3DGS's per-group learning rates (position without its schedule and scene-extent scaling).
DEFAULT_LR = {"pos": 1.6e-4, "logscale": 5e-3, "quat": 1e-3, "op_logit": 5e-2, "pmask_logit": 5e-2,
              "base": 2.5e-3, "axis": 2.5e-3, "sharp": 2.5e-3, "amp": 2.5e-3, "lmask_logit": 5e-2, "sh": 2.5e-3}


def photometric_loss(images: torch.Tensor, targets: torch.Tensor, cams: Sequence, lam: float = 0.2,
                     with_grad: bool = True):
    """(loss as a 0-d float64 tensor, dL/dimages in the flat image layout or None)."""
    lib = L.load()
    sizes = (ctypes.c_int32 * (2 * len(cams)))(*[v for c in cams for v in (int(c.width), int(c.height))])
    loss = torch.empty((), dtype=torch.float64, device="cuda")
    dl = torch.empty_like(images) if with_grad else None
    alloc = R.TorchAllocator()
    L.check(lib.megs_photometric_loss(images.data_ptr(), targets.data_ptr(), len(cams), sizes, float(lam), alloc.fn,
                                      None, loss.data_ptr(), None if dl is None else dl.data_ptr(),
                                      torch.cuda.current_stream().cuda_stream))
    loss._alloc_keepalive = alloc
    return loss, dl


class Adam:
    """Adam over a DeviceScene's planes, FP32 moments, parameters kept in their storage dtype."""

    def __init__(self, dscene: R.DeviceScene, lr: Optional[Dict[str, float]] = None, betas=(0.9, 0.999),
                 eps: float = 1e-15):
        self.ds = dscene
        self.lr = dict(DEFAULT_LR, **(lr or {}))
        self.betas = betas
        self.eps = eps
        self.step_count = 0
        self.m = {p: torch.zeros(t.shape, dtype=torch.float32, device=t.device)
                  for p, t in dscene.planes.items() if t is not None}
        self.v = {p: torch.zeros_like(m) for p, m in self.m.items()}

    def step(self, grads: Dict[str, torch.Tensor]):
        lib = L.load()
        self.step_count += 1
        s = torch.cuda.current_stream().cuda_stream
        for p, t in self.ds.planes.items():
            if t is None or grads.get(p) is None or t.numel() == 0:
                continue
            dt = R._MEGS_DT[R._group_dt(p, *self.ds.dt)]
            L.check(lib.megs_adam_step(t.numel(), t.data_ptr(), dt, grads[p].data_ptr(), self.m[p].data_ptr(),
                                       self.v[p].data_ptr(), float(self.lr[p]), float(self.betas[0]),
                                       float(self.betas[1]), float(self.eps), self.step_count, s))


def train_step(dscene: R.DeviceScene, cams: Sequence, targets: torch.Tensor, opt: Adam,
               cfg: R.Config = R.Config(), lam: float = 0.2) -> torch.Tensor:
    """Render, loss, backward, Adam: one self-contained step on the GPU; returns the loss tensor."""
    fr = R.forward(dscene, cams, cfg)
    loss, dl = photometric_loss(fr.images, targets, cams, lam)
    grads = R.backward(dscene, fr, dl)
    opt.step(grads)
    return loss

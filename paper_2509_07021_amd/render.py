"""PyTorch-facing API of the SG-splatting renderer.

PyTorch supplies device memory (through the allocation callback of the C ABI) and the current
stream; the work itself runs in libmegs.so's HIP kernels. `render` is differentiable through
`RenderFn`, a torch.autograd.Function whose backward replays the blend back to front.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L

PLANES = L.ALL_PLANES
_TORCH_DT = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}
_MEGS_DT = {"f32": L.MEGS_F32, "f16": L.MEGS_F16, "bf16": L.MEGS_BF16}
GEOM = ("pos", "logscale", "quat", "op_logit", "pmask_logit")
AMP = ("amp",)


def _group_dt(plane: str, dt_geom: str, dt_color: str, dt_amp: str) -> str:
    if plane in GEOM:
        return dt_geom
    if plane in AMP:
        return dt_amp
    return dt_color


@dataclasses.dataclass
class Config:
    tile: int = 16
    batch: int = 64
    flags: int = 0
    pair_capacity: int = 0
    waves: int = 0  # wave64s per tile workgroup (0: library default)
    subtile: int = 0  # 8: blend per 8x8 sub-tile, one independent wave each (16x16 / 32x32 tiles)

    def struct(self) -> L.MegsConfig:
        return L.MegsConfig(self.tile, self.batch, self.flags, self.waves, self.pair_capacity, self.subtile, 0)


class DeviceScene:
    """Parameter planes on the GPU (contiguous SoA torch tensors) and their storage dtypes.

    Dense lobes: axis/amp [k][3][n], sharp/lmask_logit [k][n]. Compressed rows (the post-processed
    form): lobe_off int32 [n + 1] on the device, Gaussian i owning lobes lobe_off[i] ..
    lobe_off[i + 1] - 1 (at most k), lobe planes axis/amp [3][n_lobes], sharp/lmask_logit [n_lobes].
    """

    def __init__(self, planes: dict, k: int, dt_geom="f32", dt_color="f32", dt_amp="f32",
                 lobe_off: Optional[torch.Tensor] = None, n_lobes: int = 0, keepalive=None):
        self.planes = planes
        self.k = k
        self.n = int(planes["op_logit"].shape[-1])
        self.dt = (dt_geom, dt_color, dt_amp)
        self.lobe_off = lobe_off
        self.n_lobes = int(n_lobes) if lobe_off is not None else 0
        self._keepalive = keepalive
        sh = planes.get("sh")
        self.sh_degree = 0 if sh is None else int(round(sh.shape[0] ** 0.5)) - 1
        for p in PLANES:
            t = planes.get(p)
            if t is None:
                continue
            want = _TORCH_DT[_group_dt(p, *self.dt)]
            if t.dtype != want or not t.is_contiguous() or t.device.type != "cuda":
                raise ValueError(f"plane {p}: expected a contiguous {want} CUDA tensor, got {t.dtype} on {t.device}")
        if lobe_off is not None:
            if lobe_off.dtype != torch.int32 or lobe_off.numel() != self.n + 1 or lobe_off.device.type != "cuda":
                raise ValueError("lobe_off: expected a CUDA int32 tensor of n + 1 offsets")

    @property
    def ragged(self) -> bool:
        return self.lobe_off is not None

    @classmethod
    def from_scene(cls, scene, device="cuda") -> "DeviceScene":
        """From a scenes.Scene (numpy planes; bf16 planes given as uint16 bit patterns)."""
        planes = {}
        for p in PLANES:
            a = getattr(scene, p)
            if a is None:
                planes[p] = None
                continue
            dt = _group_dt(p, scene.dt_geom, scene.dt_color, scene.dt_amp)
            if dt == "bf16":
                t = torch.from_numpy(np.ascontiguousarray(a).view(np.int16)).view(torch.bfloat16)
            else:
                t = torch.from_numpy(np.ascontiguousarray(a))
            planes[p] = t.to(device).contiguous()
        lobe_off = None
        if getattr(scene, "lobe_off", None) is not None:
            lobe_off = torch.from_numpy(np.ascontiguousarray(scene.lobe_off, dtype=np.int32)).to(device)
        return cls(planes, scene.k, scene.dt_geom, scene.dt_color, scene.dt_amp, lobe_off=lobe_off,
                   n_lobes=scene.n_lobes if lobe_off is not None else 0)

    @property
    def has_pmask(self) -> bool:
        return self.planes.get("pmask_logit") is not None

    @property
    def has_lmask(self) -> bool:
        return self.planes.get("lmask_logit") is not None

    def struct(self, planes: Optional[dict] = None) -> L.MegsScene:
        planes = planes or self.planes
        s = L.MegsScene()
        s.n, s.k = self.n, self.k
        s.dt_geom, s.dt_color, s.dt_amp = (_MEGS_DT[d] for d in self.dt)
        for p in PLANES:
            t = planes.get(p)
            setattr(s, p, None if t is None else t.data_ptr())
        s.lobe_off = None if self.lobe_off is None else self.lobe_off.data_ptr()
        s.n_lobes = self.n_lobes
        s.sh_degree = self.sh_degree
        return s

    def static_bytes(self) -> int:
        b = sum(t.numel() * t.element_size() for t in self.planes.values() if t is not None)
        return b + (0 if self.lobe_off is None else self.lobe_off.numel() * 4)


class TorchAllocator:
    """Allocation callback for the C ABI: device memory from torch's caching allocator.

    The callback closes over the block list, not over the allocator, so dropping the allocator
    frees its blocks at once (no reference cycle waiting for the garbage collector)."""

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        self.blocks = []
        blocks, dev = self.blocks, self.device

        def _alloc(ctx, nbytes):
            try:
                t = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
            except Exception:  # out of memory: the library reports MEGS_ERR_ALLOC
                return None
            blocks.append(t)
            return t.data_ptr()

        self.fn = L.ALLOC_FN(_alloc)

    def view(self, ptr: int, count: int, dtype: torch.dtype) -> torch.Tensor:
        """A tensor view of `count` elements at device address ptr inside one of the blocks."""
        if not ptr:
            raise ValueError("null pointer")
        item = torch.empty((), dtype=dtype).element_size()
        for b in self.blocks:
            base = b.data_ptr()
            if base <= ptr and ptr + count * item <= base + b.numel():
                off = ptr - base
                return b[off:off + count * item].view(dtype)
        raise ValueError("pointer not inside an allocated block")

    def nbytes(self) -> int:
        return sum(b.numel() for b in self.blocks)


def cameras_struct(cams: Sequence) -> ctypes.Array:
    arr = (L.MegsCamera * len(cams))()
    for i, c in enumerate(cams):
        m = arr[i]
        m.width, m.height = int(c.width), int(c.height)
        m.fx, m.fy, m.cx, m.cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
        R = np.asarray(c.R, np.float32).reshape(9)
        for j in range(9):
            m.R[j] = float(R[j])
        for j in range(3):
            m.t[j] = float(np.asarray(c.t, np.float32)[j])
            m.bg[j] = float(c.bg[j])
        m.znear = float(c.znear)
    return arr


def image_sizes(cams: Sequence) -> list:
    return [(int(c.height), int(c.width)) for c in cams]


def split_images(flat: torch.Tensor, cams: Sequence) -> list:
    out, off = [], 0
    for h, w in image_sizes(cams):
        out.append(flat[off:off + 3 * h * w].view(3, h, w))
        off += 3 * h * w
    return out


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Frame:
    """Result of one forward: images, the library state and the memory backing it."""

    def __init__(self, images, state, alloc, cams, cfg):
        self.images = images
        self.state = state
        self.alloc = alloc
        self.cams = cams
        self.cfg = cfg

    def buffer(self, field: str, count: int, dtype) -> torch.Tensor:
        return self.alloc.view(getattr(self.state, field), count, dtype)

    def counts(self, stream=None) -> dict:
        """The forward's counts (megs_state_counts; synchronises the stream): pairs listed, records
        culled, overflow and malformed-lobes flags."""
        c = L.MegsCounts()
        L.check(L.load().megs_state_counts(ctypes.byref(self.state), ctypes.byref(c), _stream(stream)))
        return {"pairs_needed": int(c.pairs_needed), "culled": int(c.culled), "overflow": bool(c.overflow),
                "bad_lobes": bool(c.bad_lobes)}


def forward(dscene: DeviceScene, cams: Sequence, cfg: Config = Config(), planes: Optional[dict] = None,
            stream=None) -> Frame:
    lib = L.load()
    npix = sum(h * w for h, w in image_sizes(cams))
    images = torch.empty(3 * npix, dtype=torch.float32, device="cuda")
    alloc = TorchAllocator()
    state = L.MegsState()
    sc = dscene.struct(planes)
    cam_arr = cameras_struct(cams)
    c = cfg.struct()
    L.check(lib.megs_render_forward(ctypes.byref(sc), cam_arr, len(cams), ctypes.byref(c), alloc.fn, None,
                                    images.data_ptr(), ctypes.byref(state), _stream(stream)))
    return Frame(images, state, alloc, cams, cfg)


def zero_grads_like(dscene: DeviceScene) -> dict:
    return {p: (None if t is None else torch.empty(t.shape, dtype=torch.float32, device=t.device))
            for p, t in dscene.planes.items()}


def grad_struct(grads: dict) -> L.MegsSceneGrad:
    g = L.MegsSceneGrad()
    for p in PLANES:
        t = grads.get(p)
        setattr(g, p, None if t is None else t.data_ptr())
    return g


def backward(dscene: DeviceScene, frame: Frame, dl_images: torch.Tensor, planes: Optional[dict] = None,
             stream=None) -> dict:
    """FP32 gradients of every raw plane given dL/dimage (flat, image layout)."""
    lib = L.load()
    dl = dl_images.contiguous().to(torch.float32)
    grads = zero_grads_like(dscene)
    g = grad_struct(grads)
    sc = dscene.struct(planes)
    cam_arr = cameras_struct(frame.cams)
    c = frame.cfg.struct()
    L.check(lib.megs_render_backward(ctypes.byref(sc), cam_arr, len(frame.cams), ctypes.byref(c),
                                     ctypes.byref(frame.state), dl.data_ptr(), frame.alloc.fn, None,
                                     ctypes.byref(g), _stream(stream)))
    frame.dl_keepalive = dl
    return grads


class RenderFn(torch.autograd.Function):
    """images = render(planes); backward gives dL/dplanes (FP32, cast by autograd to the plane dtype)."""

    @staticmethod
    def forward(ctx, meta, *plane_tensors):
        dscene, cams, cfg = meta
        planes = dict(zip(PLANES, plane_tensors))
        frame = forward(dscene, cams, cfg, planes=planes)
        ctx.meta = meta
        ctx.frame = frame
        ctx.planes = planes
        return frame.images

    @staticmethod
    def backward(ctx, dl):
        dscene, cams, cfg = ctx.meta
        grads = backward(dscene, ctx.frame, dl, planes=ctx.planes)
        return (None, *[grads.get(p) for p in PLANES])


def render(dscene: DeviceScene, cams: Sequence, cfg: Config = Config()) -> list:
    """Differentiable render of all views; returns one [3, H, W] tensor per view."""
    flat = RenderFn.apply((dscene, cams, cfg), *[dscene.planes.get(p) for p in PLANES])
    return split_images(flat, cams)


class Graph:
    """Batched form: forward (+ backward) of all views captured once in a hipGraph."""

    def __init__(self, dscene: DeviceScene, cams: Sequence, cfg: Config, with_backward: bool = True,
                 dl_images: Optional[torch.Tensor] = None, stream: Optional[torch.cuda.Stream] = None):
        if cfg.pair_capacity <= 0:
            raise ValueError("graph mode needs a pair capacity")
        lib = L.load()
        self.lib = lib
        self.dscene, self.cams, self.cfg = dscene, cams, cfg
        self.stream = stream or torch.cuda.Stream()
        npix = sum(h * w for h, w in image_sizes(cams))
        self.images = torch.zeros(3 * npix, dtype=torch.float32, device="cuda")
        # dL/dimage is read in place at every replay (a forward-only graph has none)
        self.dl = None
        if with_backward:
            self.dl = (dl_images.contiguous().to(torch.float32) if dl_images is not None else
                       torch.zeros(3 * npix, dtype=torch.float32, device="cuda"))
        self.grads = zero_grads_like(dscene) if with_backward else {}
        self.alloc = TorchAllocator()
        self._sc = dscene.struct()
        self._cams = cameras_struct(cams)
        self._cfg = cfg.struct()
        self._g = grad_struct(self.grads) if with_backward else None
        h = ctypes.c_void_p()
        torch.cuda.synchronize()
        L.check(lib.megs_graph_create(ctypes.byref(self._sc), self._cams, len(cams), ctypes.byref(self._cfg),
                                      self.alloc.fn, None, self.images.data_ptr(),
                                      self.dl.data_ptr() if with_backward else None,
                                      ctypes.byref(self._g) if with_backward else None, int(with_backward),
                                      self.stream.cuda_stream, ctypes.byref(h)))
        self.handle = h

    def launch(self):
        L.check(self.lib.megs_graph_launch(self.handle, self.stream.cuda_stream))

    def status(self) -> int:
        """Pairs counted at the last launch; raises MegsError on overflow."""
        n = ctypes.c_int64()
        L.check(self.lib.megs_graph_status(self.handle, ctypes.byref(n), self.stream.cuda_stream))
        return n.value

    @property
    def state(self) -> L.MegsState:
        return self.lib.megs_graph_state(self.handle).contents

    def views(self) -> list:
        return split_images(self.images, self.cams)

    def close(self):
        if getattr(self, "handle", None):
            self.lib.megs_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune_key(dscene: DeviceScene, cams: Sequence, base: Config, arch: str) -> str:
    """The cache key of an autotuning: the GPU architecture and everything about the work that the
    timings depend on (scene size, lobes, storage dtypes, masks, layout, colour model, flags, and each
    view's resolution)."""
    views = ",".join(f"{int(c.width)}x{int(c.height)}" for c in cams)
    return (f"{arch}|n={dscene.n}|k={dscene.k}|dt={'/'.join(dscene.dt)}|pmask={int(dscene.has_pmask)}"
            f"|lmask={int(dscene.has_lmask)}|ragged={int(dscene.ragged)}|sh={dscene.sh_degree if dscene.planes.get('sh') is not None else -1}"
            f"|flags={int(base.flags)}|views={views}")


def _load_cache(path: str) -> dict:
    import json
    import os
    if not path or not os.path.exists(path):
        return {}
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def _store_cache(path: str, key: str, entry: dict) -> None:
    import json
    import os
    d = _load_cache(path)
    d[key] = entry
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(dscene: DeviceScene, cams: Sequence, base: Config = Config(), reps: int = 2, dl_images=None,
             cache: Optional[str] = None, stats: Optional[dict] = None):
    """Times every (tile, waves, subtile) of AUTOTUNE_COMBOS x batch {32, 64, 128, 256}; returns
    (best Config, ms table [combo][batch]). With `cache` (a JSON file path), a result stored under
    this GPU architecture and work (autotune_key) is returned without timing (table None), and a new
    result is stored there. `stats` (a dict) receives the sweep's device memory in bytes."""
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    key = autotune_key(dscene, cams, base, arch)
    if cache:
        hit = _load_cache(cache).get(key)
        if hit:
            return Config(int(hit["tile"]), int(hit["batch"]), base.flags, base.pair_capacity, int(hit["waves"]),
                          int(hit["subtile"])), None
    lib = L.load()
    npix = sum(h * w for h, w in image_sizes(cams))
    images = torch.empty(3 * npix, dtype=torch.float32, device="cuda")
    dl = (dl_images.contiguous() if dl_images is not None else
          torch.randn(3 * npix, dtype=torch.float32, device="cuda"))
    grads = zero_grads_like(dscene)
    alloc = TorchAllocator()
    best = L.MegsConfig()
    ms = (ctypes.c_float * (len(L.AUTOTUNE_COMBOS) * len(L.AUTOTUNE_BATCHES)))()
    sc = dscene.struct()
    cam_arr = cameras_struct(cams)
    c = base.struct()
    g = grad_struct(grads)
    L.check(lib.megs_autotune(ctypes.byref(sc), cam_arr, len(cams), ctypes.byref(c), alloc.fn, None,
                              images.data_ptr(), dl.data_ptr(), ctypes.byref(g), reps, _stream(None),
                              ctypes.byref(best), ms))
    if stats is not None:
        stats["sweep_bytes"] = alloc.nbytes()
    table = np.array(list(ms), np.float32).reshape(len(L.AUTOTUNE_COMBOS), len(L.AUTOTUNE_BATCHES))
    cfg = Config(best.tile, best.batch, best.flags, best.pair_capacity, best.waves, best.subtile)
    if cache:
        _store_cache(cache, key, {"tile": cfg.tile, "batch": cfg.batch, "waves": cfg.waves, "subtile": cfg.subtile,
                                  "ms": float(table.min())})
    return cfg, table


class Profile:
    """Context manager timing each stage of eager forward/backward calls with HIP events."""

    def __enter__(self):
        L.check(L.load().megs_profile_begin())
        self.ms = {}
        self.count = {}
        return self

    def __exit__(self, *exc):
        p = L.MegsProfile()
        L.check(L.load().megs_profile_end(ctypes.byref(p)))
        self.ms = {s: p.ms[i] for i, s in enumerate(L.STAGES)}
        self.count = {s: p.count[i] for i, s in enumerate(L.STAGES)}
        return False

"""Seeded synthetic scenes and cameras for the SG-splatting renderer.

This module only draws random numbers and lays them out; it holds none of the
renderer's arithmetic. Both the GPU path and the CPU oracle take their inputs
from here, so it imports neither of them.

Parameter planes (structure of arrays, raw values as the renderer stores them):

    pos[3][N]          world position
    logscale[3][N]     per-axis log standard deviation (activated with exp)
    quat[4][N]         rotation quaternion (w, x, y, z), normalised by the renderer
    op_logit[N]        opacity logit (activated with a sigmoid)
    pmask_logit[N]     optional primitive soft-mask logit (sigmoid)
    base[3][N]         view-independent colour c0
    axis[K][3][N]      SG lobe axis (free 3-vector, normalised by the renderer)
    sharp[K][N]        SG sharpness, used as stored
    amp[K][3][N]       SG RGB amplitude
    lmask_logit[K][N]  optional per-lobe soft-mask logit (sigmoid)
    sh[M][3][N]        spherical-harmonic colour (M = (D + 1)^2, D <= 3) instead of the SG
                       planes, for the same-renderer comparison with 3DGS's colour model

The Gaussian-count range (0.2 M to 3 M) follows the primitive counts the paper
reports for its trained scenes (Appendix, table of Gaussian counts). The paper
prints no value distributions or resolutions; the draws below are the ones this
project fixes for its workloads and stand in for the paper's datasets, which are
not available here.

Draw order (PCG64, fixed): positions (cluster centres, cluster sigmas, cluster
rotations, assignments, offsets, resampling rounds), logscale, quat, op_logit,
base, axis, sharp, amp, then pmask_logit and lmask_logit when masks are on,
then camera jitter.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

PLANES = ("pos", "logscale", "quat", "op_logit", "pmask_logit",
          "base", "axis", "sharp", "amp", "lmask_logit", "sh")

# Which storage-dtype group each plane belongs to.
GEOM_PLANES = ("pos", "logscale", "quat", "op_logit", "pmask_logit")
COLOR_PLANES = ("base", "axis", "sharp", "lmask_logit", "sh")
AMP_PLANES = ("amp",)
LOBE_PLANES = ("axis", "sharp", "amp", "lmask_logit")


@dataclasses.dataclass
class Scene:
    n: int
    k: int
    pos: np.ndarray
    logscale: np.ndarray
    quat: np.ndarray
    op_logit: np.ndarray
    pmask_logit: Optional[np.ndarray]
    base: np.ndarray
    axis: np.ndarray
    sharp: np.ndarray
    amp: np.ndarray
    lmask_logit: Optional[np.ndarray]
    # storage dtype name per group: "f32", "f16" or "bf16"
    dt_geom: str = "f32"
    dt_color: str = "f32"
    dt_amp: str = "f32"
    # compressed-row lobes: None for the dense [K][...][N] lobe planes; else int32 [N + 1]
    # offsets, Gaussian i owning lobes lobe_off[i] .. lobe_off[i + 1] - 1 (at most K) of the
    # planes axis[3][L], sharp[L], amp[3][L], lmask_logit[L] (L = lobe_off[N])
    lobe_off: Optional[np.ndarray] = None
    # spherical-harmonic colour instead of SG lobes: coefficients [(D + 1)^2][3][N] (None: SG)
    sh: Optional[np.ndarray] = None

    @property
    def has_masks(self) -> bool:
        return self.pmask_logit is not None

    @property
    def ragged(self) -> bool:
        return self.lobe_off is not None

    @property
    def n_lobes(self) -> int:
        return int(self.lobe_off[-1]) if self.lobe_off is not None else self.n * self.k

    def planes(self) -> dict:
        return {p: getattr(self, p) for p in PLANES}

    def subset(self, idx: np.ndarray) -> "Scene":
        """The Gaussians idx (in the given order), same storage dtypes."""
        idx = np.asarray(idx, dtype=np.int64)
        out = {}
        lobe_off = None
        lobe_idx = None
        if self.ragged:
            cnt = np.diff(self.lobe_off.astype(np.int64))[idx]
            lobe_off = np.zeros(len(idx) + 1, np.int32)
            lobe_off[1:] = np.cumsum(cnt)
            lobe_idx = (np.repeat(self.lobe_off[:-1].astype(np.int64)[idx] - lobe_off[:-1], cnt) +
                        np.arange(int(lobe_off[-1])))
        for p in PLANES:
            a = getattr(self, p)
            if a is None:
                out[p] = None
            elif self.ragged and p in LOBE_PLANES:
                out[p] = np.ascontiguousarray(a[..., lobe_idx])
            else:
                out[p] = np.ascontiguousarray(a[..., idx])
        return Scene(n=len(idx), k=self.k, dt_geom=self.dt_geom,
                     dt_color=self.dt_color, dt_amp=self.dt_amp, lobe_off=lobe_off, **out)

    def stored(self, dt_geom="f32", dt_color="f32", dt_amp="f32") -> "Scene":
        """The same scene re-stored in reduced precision.

        f16 planes are numpy float16; bf16 planes are uint16 bit patterns
        (round to nearest even from the float32 values).
        """
        groups = {}
        for p in GEOM_PLANES:
            groups[p] = dt_geom
        for p in COLOR_PLANES:
            groups[p] = dt_color
        for p in AMP_PLANES:
            groups[p] = dt_amp
        out = {}
        for p in PLANES:
            a = getattr(self, p)
            out[p] = None if a is None else to_storage(widen(a, _dt_of(self, p)), groups[p])
        return Scene(n=self.n, k=self.k, dt_geom=dt_geom, dt_color=dt_color,
                     dt_amp=dt_amp, lobe_off=self.lobe_off, **out)

    def widened(self) -> dict:
        """All planes as float64 holding exactly the stored values (plus "lobe_off" for
        compressed-row scenes)."""
        out = {p: (None if getattr(self, p) is None else
                   widen(getattr(self, p), _dt_of(self, p)).astype(np.float64))
               for p in PLANES}
        if self.ragged:
            out["lobe_off"] = np.ascontiguousarray(self.lobe_off, dtype=np.int32)
        return out


def _dt_of(scene: Scene, plane: str) -> str:
    if plane in GEOM_PLANES:
        return scene.dt_geom
    if plane in AMP_PLANES:
        return scene.dt_amp
    return scene.dt_color


def to_storage(a32: np.ndarray, dt: str) -> np.ndarray:
    a32 = np.ascontiguousarray(a32, dtype=np.float32)
    if dt == "f32":
        return a32
    if dt == "f16":
        return a32.astype(np.float16)
    if dt == "bf16":
        bits = a32.view(np.uint32).astype(np.uint64)
        rounded = (bits + 0x7FFF + ((bits >> 16) & 1)) >> 16
        return rounded.astype(np.uint16)
    raise ValueError(dt)


def widen(a: np.ndarray, dt: str) -> np.ndarray:
    """Stored values to float32 (exact for f16 and bf16)."""
    if dt == "f32":
        return np.asarray(a, dtype=np.float32)
    if dt == "f16":
        return np.asarray(a, dtype=np.float16).astype(np.float32)
    if dt == "bf16":
        return (np.asarray(a, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)
    raise ValueError(dt)


@dataclasses.dataclass
class Camera:
    """Pinhole camera, OpenCV axes (x right, y down, z forward).

    R, t map world to camera: x_cam = R @ x_world + t. Pixel (i, j) has its
    centre at (i + 0.5, j + 0.5). All values are float32 as the renderer
    receives them.
    """
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray  # (3, 3) float32, row-major
    t: np.ndarray  # (3,) float32
    znear: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)

    def as_f32(self) -> "Camera":
        f = lambda v: float(np.float32(v))
        return Camera(self.width, self.height, f(self.fx), f(self.fy), f(self.cx), f(self.cy),
                      np.asarray(self.R, np.float32), np.asarray(self.t, np.float32),
                      f(self.znear), tuple(f(b) for b in self.bg))


def look_at(eye, width: int, height: int, fov_y_deg: float = 60.0,
            target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0), bg=(0.0, 0.0, 0.0)) -> Camera:
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    upv = np.asarray(up, np.float64)
    if abs(float(f @ upv)) > 0.999:
        upv = np.array([0.0, 1.0, 0.0])
    x = np.cross(f, upv)
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    R = np.stack([x, y, f])
    t = -R @ eye
    foc = (height / 2.0) / math.tan(math.radians(fov_y_deg) / 2.0)
    return Camera(width, height, foc, foc, width / 2.0, height / 2.0,
                  R.astype(np.float32), t.astype(np.float32), 0.2, tuple(bg)).as_f32()


def crop_camera(cam: Camera, width: int, height: int) -> Camera:
    """The centred width x height window of cam's image, same focal length."""
    return Camera(width, height, cam.fx, cam.fy,
                  cam.cx - (cam.width - width) / 2.0, cam.cy - (cam.height - height) / 2.0,
                  cam.R.copy(), cam.t.copy(), cam.znear, cam.bg).as_f32()


def _uniform_positions(rng, n):
    return rng.uniform(-1.0, 1.0, size=(3, n))


def _clustered_positions(rng, n, n_clusters=32, box=3.0):
    centres = rng.uniform(-box, box, size=(n_clusters, 3))
    sigmas = rng.uniform(0.05, 0.3, size=(n_clusters, 3))
    rots = []
    for _ in range(n_clusters):
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        q = q * np.sign(np.diag(r))[None, :]
        if np.linalg.det(q) < 0:
            q[:, 0] = -q[:, 0]
        rots.append(q)
    rots = np.stack(rots)
    assign = rng.integers(0, n_clusters, size=n)
    z = rng.standard_normal((n, 3))
    pts = centres[assign] + np.einsum("nij,nj->ni", rots[assign], sigmas[assign] * z)
    bad = np.nonzero(np.any(np.abs(pts) > box, axis=1))[0]
    while bad.size:
        zb = rng.standard_normal((bad.size, 3))
        a = assign[bad]
        pts[bad] = centres[a] + np.einsum("nij,nj->ni", rots[a], sigmas[a] * zb)
        bad = bad[np.any(np.abs(pts[bad]) > box, axis=1)]
    return pts.T


def _normalise(a, axis):
    return a / np.linalg.norm(a, axis=axis, keepdims=True)


def make_scene(n: int, k: int, seed: int, clustered: bool, masks: bool) -> Scene:
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = _clustered_positions(rng, n) if clustered else _uniform_positions(rng, n)
    logscale = rng.normal(-3.5, 0.5, size=(3, n))
    quat = _normalise(rng.standard_normal((4, n)), 0)
    op_logit = rng.normal(0.0, 1.0, size=n)
    base = rng.uniform(0.0, 1.0, size=(3, n))
    axis = _normalise(rng.standard_normal((k, 3, n)), 1)
    sharp = np.exp(rng.uniform(0.0, math.log(50.0), size=(k, n)))
    amp = rng.normal(0.0, 0.2, size=(k, 3, n))
    pm = lm = None
    if masks:
        pm = rng.normal(1.0, 1.5, size=n)
        lm = rng.normal(0.5, 1.5, size=(k, n))
    f32 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float32)
    return Scene(n=n, k=k, pos=f32(pos), logscale=f32(logscale), quat=f32(quat),
                 op_logit=f32(op_logit), pmask_logit=f32(pm), base=f32(base),
                 axis=f32(axis), sharp=f32(sharp), amp=f32(amp), lmask_logit=f32(lm))


@dataclasses.dataclass(frozen=True)
class Workload:
    """A named workload: scene recipe, cameras and tile size."""
    name: str
    n: int
    k: int
    clustered: bool
    masks: bool
    seed: int
    cameras: str            # "front4", "sphere6", "ring16", "ring8"
    resolution: tuple = (128, 128)
    tile: int = 16
    storage: tuple = ("f32", "f32", "f32")
    description: str = ""
    recipe: str = "plain"   # "post_admm": post_admm() applied to the plain scene


WORKLOADS = {
    "small_2k_128px": Workload(
        "small_2k_128px", 2000, 3, False, False, 1, "front4", (128, 128), 16,
        description="2,000 uniform Gaussians, 3 lobes, 1 view 128x128, FP32"),
    "clustered_200k_720p": Workload(
        "clustered_200k_720p", 200_000, 4, True, False, 2, "sphere6", (1280, 720), 16,
        description="200k clustered Gaussians, 4 lobes, 1 view 1280x720, FP32"),
    "masked_1m_1080p": Workload(
        "masked_1m_1080p", 1_000_000, 4, True, True, 3, "sphere6", (1920, 1080), 16,
        description="1M clustered Gaussians, 4 lobes, soft masks, 1 view 1920x1080, FP32"),
    "batched_500k_16views": Workload(
        "batched_500k_16views", 500_000, 4, True, False, 4, "ring16", (0, 0), 16,
        description="500k clustered Gaussians, 4 lobes, 16 views 360p-1080p, FP32"),
    "post_admm_1600k_1080p": Workload(
        "post_admm_1600k_1080p", 1_600_000, 3, True, True, 6, "sphere6", (1920, 1080), 16,
        recipe="post_admm",
        description="1.6M clustered Gaussians, 3 lobes, soft masks, as left by the memory-constrained "
                    "optimisation (40% near-zero opacity, 68% of lobes with sharpness < 1); compacted "
                    "to about 0.96M Gaussians with 0-3 lobes, 1 view 1920x1080, FP32"),
    "fp16_3m_8x1080p": Workload(
        "fp16_3m_8x1080p", 3_000_000, 4, True, False, 5, "ring8", (1920, 1080), 16,
        storage=("f16", "f16", "bf16"),
        description="3M clustered Gaussians, 4 lobes, FP16 storage (BF16 amplitudes), 8 views 1920x1080"),
}

RING16_RES = ((640, 360), (960, 540), (1280, 720), (1920, 1080))


def make_cameras(w: Workload) -> list:
    rng = np.random.Generator(np.random.PCG64(w.seed + 1000))
    if w.cameras == "front4":
        return [look_at((0.0, -4.0, 0.0), *w.resolution)]
    if w.cameras == "sphere6":
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        return [look_at(6.0 * u, *w.resolution)]
    if w.cameras in ("ring16", "ring8"):
        nv = 16 if w.cameras == "ring16" else 8
        cams = []
        for i in range(nv):
            az = 2.0 * math.pi * i / nv
            el = math.radians(rng.uniform(-15.0, 15.0))
            eye = 6.0 * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
            res = RING16_RES[i % 4] if w.cameras == "ring16" else w.resolution
            cams.append(look_at(eye, *res))
        return cams
    raise ValueError(w.cameras)


def ring_cameras(nv: int, seed: int, resolution=(1920, 1080), radius: float = 6.0) -> list:
    """nv cameras on a ring of the given radius around the origin, elevation jittered by up to
    15 degrees (seeded), all at one resolution."""
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    cams = []
    for i in range(nv):
        az = 2.0 * math.pi * i / nv
        el = math.radians(rng.uniform(-15.0, 15.0))
        eye = radius * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
        cams.append(look_at(eye, *resolution))
    return cams


def make_workload(name: str, n: Optional[int] = None):
    """(scene, cameras) for a named workload; n overrides the Gaussian count."""
    w = WORKLOADS[name]
    if n is not None:
        w = dataclasses.replace(w, n=n)
    scene = make_scene(w.n, w.k, w.seed, w.clustered, w.masks)
    if w.recipe == "post_admm":
        scene = post_admm(scene, w.seed)
    if w.storage != ("f32", "f32", "f32"):
        scene = scene.stored(*w.storage)
    return scene, make_cameras(w)


def random_scene(rng: np.random.Generator, n: int, k: int, masks: bool,
                 spread: float = 1.0, logscale_mu: float = -2.0) -> Scene:
    """Small random scene for property tests (positions in a box of half-width spread)."""
    pos = rng.uniform(-spread, spread, size=(3, n))
    logscale = rng.normal(logscale_mu, 0.5, size=(3, n))
    quat = _normalise(rng.standard_normal((4, n)), 0)
    op_logit = rng.normal(0.5, 1.0, size=n)
    base = rng.uniform(0.0, 1.0, size=(3, n))
    axis = _normalise(rng.standard_normal((k, 3, n)), 1)
    sharp = np.exp(rng.uniform(0.0, math.log(50.0), size=(k, n)))
    amp = rng.normal(0.0, 0.2, size=(k, 3, n))
    pm = rng.normal(1.0, 1.5, size=n) if masks else None
    lm = rng.normal(0.5, 1.5, size=(k, n)) if masks else None
    f32 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float32)
    return Scene(n=n, k=k, pos=f32(pos), logscale=f32(logscale), quat=f32(quat),
                 op_logit=f32(op_logit), pmask_logit=f32(pm), base=f32(base),
                 axis=f32(axis), sharp=f32(sharp), amp=f32(amp), lmask_logit=f32(lm))


def ragged_scene(rng: np.random.Generator, n: int, kmax: int, masks: bool,
                 spread: float = 1.0, logscale_mu: float = -2.0) -> Scene:
    """Small random compressed-row scene: each Gaussian draws 0..kmax lobes (uniform), lobes
    drawn like random_scene's. Draw order: the dense fields of random_scene with k = 0, then the
    lobe counts, axis, sharp, amp and (with masks) the lobe mask logits."""
    sc = random_scene(rng, n, 0, masks, spread, logscale_mu)
    cnt = rng.integers(0, kmax + 1, size=n)
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(cnt)
    nl = int(off[-1])
    axis = _normalise(rng.standard_normal((3, nl)), 0)
    sharp = np.exp(rng.uniform(0.0, math.log(50.0), size=nl))
    amp = rng.normal(0.0, 0.2, size=(3, nl))
    lm = rng.normal(0.5, 1.5, size=nl) if masks else None
    f32 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float32)
    return dataclasses.replace(sc, k=kmax, axis=f32(axis), sharp=f32(sharp), amp=f32(amp), lmask_logit=f32(lm),
                               lobe_off=off.astype(np.int32))


def post_admm(scene: Scene, seed: int, prim_frac: float = 0.4, lobe_frac: float = 0.68) -> Scene:
    """The state the memory-constrained optimisation leaves behind (Sec. 3.3, post-processing
    procedure: many Gaussians with near-zero opacity and many lobes with near-zero sharpness),
    imposed on a dense scene: a prim_frac share of Gaussians gets opacity logits N(-9, 1)
    (opacity about 1e-4, below any sensible threshold) and a lobe_frac share of lobes gets
    sharpness U(0, 1) (below the paper's lobe threshold of 1). With K = 3 lobes and the default
    0.68, the lobes that survive average 0.96 per Gaussian, i.e. 3 + 7 x 0.96 = 9.7 colour floats
    (the paper's per-Gaussian colour cost after post-processing). Draw order: the Gaussian
    choice, its logits, the lobe choice, its sharpness."""
    rng = np.random.Generator(np.random.PCG64(seed + 2000))
    op = scene.op_logit.astype(np.float32).copy()
    sharp = scene.sharp.astype(np.float32).copy()
    pick = rng.random(scene.n) < prim_frac
    op[pick] = rng.normal(-9.0, 1.0, size=int(pick.sum()))
    lpick = rng.random(sharp.shape) < lobe_frac
    sharp[lpick] = rng.uniform(0.0, 1.0, size=int(lpick.sum()))
    return dataclasses.replace(scene, op_logit=op, sharp=sharp)


def sh_scene(scene: Scene, seed: int, degree: int = 3) -> Scene:
    """The scene's geometry with spherical-harmonic colour of the given degree instead of SG
    lobes: DC coefficients U(-1, 1.8), higher coefficients N(0, 0.1^2) (seeded; draw order: the
    DC plane, then coefficients 1.. in plane order)."""
    rng = np.random.Generator(np.random.PCG64(seed + 3000))
    m = (degree + 1) ** 2
    sh = np.zeros((m, 3, scene.n), np.float64)
    sh[0] = rng.uniform(-1.0, 1.8, size=(3, scene.n))
    sh[1:] = rng.normal(0.0, 0.1, size=(m - 1, 3, scene.n))
    empty = lambda *shape: np.zeros(shape, np.float32)
    sh = to_storage(sh.astype(np.float32), scene.dt_color)
    return dataclasses.replace(scene, k=0, base=None, axis=empty(0, 3, scene.n), sharp=empty(0, scene.n),
                               amp=to_storage(empty(0, 3, scene.n), scene.dt_amp), lmask_logit=None, lobe_off=None,
                               sh=sh)


def axis_nearest(scene: Scene, cam: Camera, count: int) -> np.ndarray:
    """Indices of the count Gaussians angularly nearest the camera's optical axis,
    in ascending index order (used to cut a small crop out of a large scene)."""
    pos = widen(scene.pos, scene.dt_geom).astype(np.float64)
    R = cam.R.astype(np.float64)
    eye = -R.T @ cam.t.astype(np.float64)
    rel = pos - eye[:, None]
    fwd = R[2]
    cosang = (fwd @ rel) / np.linalg.norm(rel, axis=0)
    idx = np.argsort(-cosang, kind="stable")[:count]
    return np.sort(idx)


def loss_weights(cams: Sequence[Camera], seed: int) -> list:
    """Seeded N(0, 1) weights w per view, shaped [3][H][W], for L = sum(w * image)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [rng.standard_normal((3, c.height, c.width)).astype(np.float32) for c in cams]

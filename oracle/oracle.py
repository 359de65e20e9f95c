"""Python driver for the FP64 CPU oracle (megs_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline use it; the renderer never does. It imports nothing from the renderer
package; its inputs are the seeded scenes (as float64 planes holding the exact
stored values) and cameras.

The C file does the arithmetic; this module builds and loads it, marshals
arrays, and composes the per-view steps into a whole multi-view render and its
gradient, plus a central finite-difference harness.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "megs_oracle.c")
LIB = os.path.join(HERE, "libmegs_oracle.so")

SCENE_PLANES = ("pos", "logscale", "quat", "op_logit", "pmask_logit",
                "base", "axis", "sharp", "amp", "lmask_logit")
PLANES = SCENE_PLANES + ("sh",)   # "sh": spherical-harmonic coefficients [(D + 1)^2][3][n] (SH colour)

_dp = ctypes.POINTER(ctypes.c_double)


class OScene(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("k", ctypes.c_int32), ("pad", ctypes.c_int32)] + \
               [(p, _dp) for p in SCENE_PLANES] + [("lobe_off", ctypes.POINTER(ctypes.c_int32)),
                                                    ("n_lobes", ctypes.c_int64), ("sh", _dp),
                                                    ("sh_degree", ctypes.c_int32), ("pad2", ctypes.c_int32)]


class OCam(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("R", ctypes.c_double * 9), ("t", ctypes.c_double * 3),
                ("znear", ctypes.c_double), ("bg", ctypes.c_double * 3)]


class OGrad(ctypes.Structure):
    _fields_ = [(p, _dp) for p in PLANES]


# MEGS_ORACLE_SANITIZE=1 builds and loads a separate copy instrumented with AddressSanitizer and
# UndefinedBehaviorSanitizer that stops at the first report (the sanitizer pin run; the process must
# preload the sanitizer runtimes).
SANITIZE = os.environ.get("MEGS_ORACLE_SANITIZE", "") == "1"
if SANITIZE:
    LIB = os.path.join(HERE, "libmegs_oracle_san.so")
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        opt = SAN_FLAGS if SANITIZE else ["-O2"]
        subprocess.check_call(["gcc", *opt, "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-std=c11", "-Wall", "-shared", "-fPIC", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        vp = ctypes.c_void_p
        L.oracle_threads.restype = ctypes.c_int32
        L.oracle_project.argtypes = [ctypes.POINTER(OScene), ctypes.POINTER(OCam), ctypes.c_int32, vp, vp]
        L.oracle_sg_color.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp]
        L.oracle_sg_color_many.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp, ctypes.c_int64, vp, vp]
        L.oracle_pairs.argtypes = [ctypes.c_int64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                   ctypes.c_int32, ctypes.c_int64, vp, vp, vp]
        L.oracle_pairs.restype = ctypes.c_int64
        L.oracle_tile_candidates.argtypes = [ctypes.c_int64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                             ctypes.c_int32, ctypes.c_double, vp, vp, vp]
        L.oracle_tile_candidates.restype = ctypes.c_int64
        L.oracle_box_min.argtypes = [ctypes.c_int64, vp, vp, vp, vp, vp]
        L.oracle_sort_pairs.argtypes = [ctypes.c_int64, vp, vp, ctypes.c_int64, vp]
        L.oracle_subtile_flags.argtypes = [ctypes.c_int64, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int32, vp, vp, vp,
                                           ctypes.c_int32, ctypes.c_double, vp, vp]
        L.oracle_blend.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp,
                                   vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int64, vp]
        L.oracle_blend.restype = ctypes.c_int64
        L.oracle_bruteforce.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_int64, vp,
                                        vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.oracle_blend_backward.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp,
                                            vp, vp, vp, vp, vp, vp, vp, ctypes.c_int64, vp,
                                            ctypes.c_int32, vp, vp]
        L.oracle_project_backward.argtypes = [ctypes.POINTER(OScene), ctypes.POINTER(OCam), ctypes.c_int32,
                                              vp, ctypes.POINTER(OGrad)]
        L.oracle_sh_basis.argtypes = [ctypes.c_int64, vp, vp, vp]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def make_oscene(planes: dict, k: int):
    """planes: float64 arrays (exact stored values), plus int32 "lobe_off" [n + 1] for the
    compressed-row lobe layout. Returns (struct, keepalive)."""
    keep = {p: _c64(planes.get(p)) for p in PLANES}
    n = keep["op_logit"].shape[0]
    s = OScene(n=n, k=k, pad=0)
    for p in PLANES:
        setattr(s, p, None if keep[p] is None else keep[p].ctypes.data_as(_dp))
    if keep["sh"] is not None:
        nm = keep["sh"].shape[0]
        s.sh_degree = int(round(nm ** 0.5)) - 1
        assert (s.sh_degree + 1) ** 2 == nm and 0 <= s.sh_degree <= 3, "sh planes must be [(D + 1)^2][3][n], D <= 3"
    off = planes.get("lobe_off")
    if off is not None:
        off = np.ascontiguousarray(off, dtype=np.int32)
        keep["lobe_off"] = off
        s.lobe_off = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        s.n_lobes = int(off[-1])
    return s, keep


def make_ocam(cam) -> OCam:
    c = OCam()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = np.asarray(cam.R, np.float64).reshape(9)
    for i in range(9):
        c.R[i] = R[i]
    for i in range(3):
        c.t[i] = float(np.asarray(cam.t, np.float64)[i])
        c.bg[i] = float(cam.bg[i])
    c.znear = float(cam.znear)
    return c


def project(planes: dict, k: int, cam, tile: int) -> dict:
    """FP64 records of all Gaussians in one view."""
    s, keep = make_oscene(planes, k)
    n = s.n
    f = np.zeros((n, 11), np.float64)
    i = np.zeros((n, 7), np.int32)
    c = make_ocam(cam)
    lib().oracle_project(ctypes.byref(s), ctypes.byref(c), tile, _ptr(f), _ptr(i))
    return {"u": f[:, 0].copy(), "v": f[:, 1].copy(), "depth": f[:, 2].copy(),
            "conic": f[:, 3:6].copy(), "o": f[:, 6].copy(), "rgb": f[:, 7:10].copy(), "cutoff": f[:, 10].copy(),
            "valid": i[:, 0].copy(), "radius": i[:, 1].copy(), "rect": i[:, 2:6].copy(),
            "ntiles": i[:, 6].copy()}


def sg_color(base, axis, sharp, amp, direction, mask=None) -> np.ndarray:
    base = _c64(base); axis = _c64(axis); sharp = _c64(sharp); amp = _c64(amp)
    direction = _c64(direction)
    mask = _c64(mask)
    out = np.zeros(3, np.float64)
    lib().oracle_sg_color(len(sharp), _ptr(base), _ptr(axis), _ptr(sharp), _ptr(amp), _ptr(mask),
                          _ptr(direction), _ptr(out))
    return out


def sg_color_many(base, axis, sharp, amp, directions, mask=None) -> np.ndarray:
    """SG colour for many directions [m][3] -> [m][3]."""
    base = _c64(base); axis = _c64(axis); sharp = _c64(sharp); amp = _c64(amp)
    d = _c64(directions)
    mask = _c64(mask)
    out = np.zeros((len(d), 3), np.float64)
    lib().oracle_sg_color_many(len(sharp), _ptr(base), _ptr(axis), _ptr(sharp), _ptr(amp), _ptr(mask),
                               len(d), _ptr(d), _ptr(out))
    return out


def sh_basis(dirs):
    """Real spherical harmonics of degree <= 3 at unit directions dirs [m][3]: (Y [m][16],
    dY/d(x, y, z) [m][16][3])."""
    dirs = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    Y = np.zeros((len(dirs), 16))
    dY = np.zeros((len(dirs), 16, 3))
    lib().oracle_sh_basis(len(dirs), _ptr(dirs), _ptr(Y), _ptr(dY))
    return Y, dY


def threads() -> int:
    return int(lib().oracle_threads())


def tile_layout(cams: Sequence, tile: int):
    """Per-view tile counts and the global tile offset of each view."""
    counts = [((c.width + tile - 1) // tile) * ((c.height + tile - 1) // tile) for c in cams]
    off = np.zeros(len(cams) + 1, np.int64)
    off[1:] = np.cumsum(counts)
    return off


def _view_arrays(cams, tile):
    w = np.array([c.width for c in cams], np.int32)
    h = np.array([c.height for c in cams], np.int32)
    return w, h, tile_layout(cams, tile)


def pairs(u, v, depth_f32, radius, conic, cutoff, valid, rec_view, cams, tile: int):
    """Sorted key table over records of several views.

    u, v: float64 means; depth_f32: float32 depths; radius, valid, rec_view: int32; conic [n][3]
    and cutoff [n] (float64): a tile of a record's rectangle is listed when the minimum of the
    record's quadratic form over the tile's pixel-centre box is <= cutoff.
    Returns keys (uint64), vals (uint32), ranges ([T][2] uint32), tile offsets.
    """
    u = _c64(u); v = _c64(v)
    cn = _c64(conic); cu = _c64(cutoff)
    d = np.ascontiguousarray(depth_f32, np.float32)
    r = np.ascontiguousarray(radius, np.int32)
    va = np.ascontiguousarray(valid, np.int32)
    rv = np.ascontiguousarray(rec_view, np.int32)
    w, h, off = _view_arrays(cams, tile)
    total = int(off[-1])
    L = lib()
    n = len(u)
    cnt = L.oracle_pairs(n, _ptr(u), _ptr(v), _ptr(d), _ptr(r), _ptr(cn), _ptr(cu), _ptr(va), _ptr(rv), _ptr(w),
                         _ptr(h), _ptr(off), tile, total, None, None, None)
    keys = np.zeros(max(cnt, 1), np.uint64)
    vals = np.zeros(max(cnt, 1), np.uint32)
    ranges = np.zeros((total, 2), np.uint32)
    L.oracle_pairs(n, _ptr(u), _ptr(v), _ptr(d), _ptr(r), _ptr(cn), _ptr(cu), _ptr(va), _ptr(rv), _ptr(w), _ptr(h),
                   _ptr(off), tile, total, _ptr(keys), _ptr(vals), _ptr(ranges))
    return keys[:cnt], vals[:cnt], ranges, off


def tile_candidates(u, v, radius, conic, cutoff, valid, rec_view, cams, tile: int, band: float):
    """Every (tile, record) pair of the records' rectangles that is listed or whose decision lies within
    the relative band of the level: (global tile int64, record uint32, state uint8: 1 listed, 2 within
    the band), in record order."""
    u = _c64(u); v = _c64(v)
    cn = _c64(conic); cu = _c64(cutoff)
    r = np.ascontiguousarray(radius, np.int32)
    va = np.ascontiguousarray(valid, np.int32)
    rv = np.ascontiguousarray(rec_view, np.int32)
    w, h, off = _view_arrays(cams, tile)
    L = lib()
    args = (len(u), _ptr(u), _ptr(v), _ptr(r), _ptr(cn), _ptr(cu), _ptr(va), _ptr(rv), _ptr(w), _ptr(h), _ptr(off),
            tile, float(band))
    cnt = L.oracle_tile_candidates(*args, None, None, None)
    tl = np.zeros(max(cnt, 1), np.int64)
    rc = np.zeros(max(cnt, 1), np.uint32)
    st = np.zeros(max(cnt, 1), np.uint8)
    L.oracle_tile_candidates(*args, _ptr(tl), _ptr(rc), _ptr(st))
    return tl[:cnt], rc[:cnt], st[:cnt]


def box_min(u, v, conic, box) -> np.ndarray:
    """min over each box [x0, x1] x [y0, y1] of (p - m)' C (p - m) (-inf for a conic that is not positive
    definite). u, v: [m]; conic: [m][3] = (a, b, c); box: [m][4]."""
    u = _c64(np.atleast_1d(u)); v = _c64(np.atleast_1d(v))
    cn = _c64(np.reshape(conic, (-1, 3))); bx = _c64(np.reshape(box, (-1, 4)))
    out = np.zeros(len(u))
    lib().oracle_box_min(len(u), _ptr(u), _ptr(v), _ptr(cn), _ptr(bx), _ptr(out))
    return out


def sort_pairs(keys, vals, total_tiles: int):
    """(keys, vals) ordered by (key, value) and the per-tile [start, end) ranges."""
    keys = np.array(keys, np.uint64, copy=True)
    vals = np.array(vals, np.uint32, copy=True)
    ranges = np.zeros((int(total_tiles), 2), np.uint32)
    lib().oracle_sort_pairs(len(keys), _ptr(keys), _ptr(vals), int(total_tiles), _ptr(ranges))
    return keys, vals, ranges


def subtile_flags(tiles, recs, u, v, conic, cutoff, rec_view, cams, tile: int, band: float):
    """For each listed pair, the 8 x 8 sub-tiles of the tile (bit r S + c, S = tile / 8) whose pixel-centre
    boxes the record's ellipse reaches: (set uint32, near uint32), near = within the relative band."""
    tiles = np.ascontiguousarray(tiles, np.int64)
    recs = np.ascontiguousarray(recs, np.uint32)
    u = _c64(u); v = _c64(v)
    cn = _c64(conic); cu = _c64(cutoff)
    rv = np.ascontiguousarray(rec_view, np.int32)
    w, h, off = _view_arrays(cams, tile)
    s = np.zeros(len(tiles), np.uint32)
    nb = np.zeros(len(tiles), np.uint32)
    lib().oracle_subtile_flags(len(tiles), _ptr(tiles), _ptr(recs), _ptr(u), _ptr(v), _ptr(cn), _ptr(cu), _ptr(rv),
                               len(cams), _ptr(w), _ptr(h), _ptr(off), tile, float(band), _ptr(s), _ptr(nb))
    return s, nb


def _recs(rec):
    return (_c64(rec["u"]), _c64(rec["v"]), _c64(rec["conic"]), _c64(rec["o"]), _c64(rec["rgb"]))


def blend(cam, tile: int, rec: dict, vals, ranges_view, importance=None):
    """Tiled forward blend of one view. ranges_view: the view's [T_v][2] slice. When importance
    (float64 [records]) is given, each record's blending weights are added into it."""
    u, v, conic, o, rgb = _recs(rec)
    w, h = cam.width, cam.height
    bg = np.asarray(cam.bg, np.float64)
    image = np.zeros((3, h, w), np.float64)
    T = np.zeros((h, w), np.float64)
    last = np.zeros((h, w), np.int32)
    flag = np.zeros((h, w), np.int32)
    sig = np.zeros((h, w), np.uint64)
    vals = np.ascontiguousarray(vals, np.uint32)
    rv = np.ascontiguousarray(ranges_view, np.uint32)
    nfrag = lib().oracle_blend(w, h, tile, _ptr(bg), _ptr(u), _ptr(v), _ptr(conic), _ptr(o), _ptr(rgb),
                               _ptr(vals), _ptr(rv), _ptr(image), _ptr(T), _ptr(last), _ptr(flag), _ptr(sig),
                               len(vals), _ptr(importance))
    return {"image": image, "T": T, "last": last, "flag": flag, "sig": sig, "nfrag": int(nfrag)}


def bruteforce(cam, rec: dict, valid):
    u, v, conic, o, rgb = _recs(rec)
    depth = _c64(rec["depth"])
    va = np.ascontiguousarray(valid, np.int32)
    w, h = cam.width, cam.height
    bg = np.asarray(cam.bg, np.float64)
    image = np.zeros((3, h, w), np.float64)
    T = np.zeros((h, w), np.float64)
    last = np.zeros((h, w), np.int32)
    flag = np.zeros((h, w), np.int32)
    lib().oracle_bruteforce(w, h, _ptr(bg), len(u), _ptr(va), _ptr(depth), _ptr(u), _ptr(v), _ptr(conic),
                            _ptr(o), _ptr(rgb), _ptr(image), _ptr(T), _ptr(last), _ptr(flag))
    return {"image": image, "T": T, "last": last, "flag": flag}


def blend_backward(cam, tile: int, rec: dict, vals, ranges_view, dl, direct: bool = False, grad2d=None,
                   grad2d_abs=None):
    """Per-record 2D gradients [n][9] for one view (added into grad2d if given; the sums of the
    contributions' absolute values are added into grad2d_abs when given)."""
    u, v, conic, o, rgb = _recs(rec)
    n = len(u)
    if grad2d is None:
        grad2d = np.zeros((n, 9), np.float64)
    bg = np.asarray(cam.bg, np.float64)
    vals = np.ascontiguousarray(vals, np.uint32)
    rv = np.ascontiguousarray(ranges_view, np.uint32)
    dl = _c64(dl)
    lib().oracle_blend_backward(cam.width, cam.height, tile, _ptr(bg), _ptr(u), _ptr(v), _ptr(conic), _ptr(o),
                                _ptr(rgb), _ptr(vals), _ptr(rv), len(vals), _ptr(dl), int(direct), _ptr(grad2d),
                                _ptr(grad2d_abs))
    return grad2d


def zero_grads(planes: dict) -> dict:
    return {p: (None if planes.get(p) is None else np.zeros_like(_c64(planes[p]))) for p in PLANES}


def project_backward(planes: dict, k: int, cam, tile: int, grad2d, grads: dict):
    """Adds one view's raw-parameter gradients into grads (float64 planes)."""
    s, keep = make_oscene(planes, k)
    g = OGrad()
    for p in PLANES:
        setattr(g, p, None if grads[p] is None else grads[p].ctypes.data_as(_dp))
    c = make_ocam(cam)
    g2 = _c64(grad2d)
    lib().oracle_project_backward(ctypes.byref(s), ctypes.byref(c), tile, _ptr(g2), ctypes.byref(g))
    return grads


def render(planes: dict, k: int, cams: Sequence, tile: int) -> dict:
    """Whole FP64 multi-view forward: per-view records, key table, blend."""
    n = len(planes["op_logit"])
    recs = [project(planes, k, c, tile) for c in cams]
    cat = lambda key: np.concatenate([r[key] for r in recs])
    rec_all = {key: cat(key) for key in ("u", "v", "depth", "conic", "o", "rgb", "cutoff", "valid", "radius",
                                         "ntiles")}
    rec_view = np.repeat(np.arange(len(cams), dtype=np.int32), n)
    keys, vals, ranges, off = pairs(rec_all["u"], rec_all["v"], rec_all["depth"].astype(np.float32),
                                    rec_all["radius"], rec_all["conic"], rec_all["cutoff"], rec_all["valid"],
                                    rec_view, cams, tile)
    views = []
    for vi, c in enumerate(cams):
        views.append(blend(c, tile, rec_all, vals, ranges[off[vi]:off[vi + 1]]))
    return {"records": rec_all, "per_view_records": recs, "keys": keys, "vals": vals, "ranges": ranges,
            "tile_off": off, "views": views, "images": [vw["image"] for vw in views]}


def render_backward(planes: dict, k: int, cams: Sequence, tile: int, dl_images: Sequence, fwd: dict = None):
    """Gradients of L = sum(dl_images[v] * image_v) with respect to every raw plane."""
    if fwd is None:
        fwd = render(planes, k, cams, tile)
    n = len(planes["op_logit"])
    grads = zero_grads(planes)
    grad2d = np.zeros((n * len(cams), 9), np.float64)
    off = fwd["tile_off"]
    for vi, c in enumerate(cams):
        blend_backward(c, tile, fwd["records"], fwd["vals"], fwd["ranges"][off[vi]:off[vi + 1]],
                       dl_images[vi], grad2d=grad2d)
    for vi, c in enumerate(cams):
        project_backward(planes, k, c, tile, grad2d[vi * n:(vi + 1) * n], grads)
    return grads, grad2d


def loss(planes: dict, k: int, cams, tile: int, weights) -> tuple:
    fwd = render(planes, k, cams, tile)
    L = sum(float(np.sum(w.astype(np.float64) * img)) for w, img in zip(weights, fwd["images"]))
    sig = tuple(np.concatenate([vw["sig"].ravel() for vw in fwd["views"]]).tolist())
    return L, hash(sig)


def fd_gradient(planes: dict, k: int, cams, tile: int, weights, plane: str, flat_indices, rel_h: float = 1e-6):
    """Central differences of L for chosen entries of one plane.

    Returns (fd values, mask of entries whose +-h perturbation kept every per-pixel
    decision -- the included fragment set and clamp states -- unchanged)."""
    _, sig0 = loss(planes, k, cams, tile, weights)
    out = np.zeros(len(flat_indices))
    ok = np.ones(len(flat_indices), bool)
    for j, fi in enumerate(flat_indices):
        base = {p: (None if planes.get(p) is None else np.array(planes[p], np.float64, copy=True)) for p in PLANES}
        if planes.get("lobe_off") is not None:
            base["lobe_off"] = planes["lobe_off"]
        arr = base[plane].reshape(-1)
        x0 = arr[fi]
        h = rel_h * max(1.0, abs(x0))
        arr[fi] = x0 + h
        Lp, sp = loss(base, k, cams, tile, weights)
        arr[fi] = x0 - h
        Lm, sm = loss(base, k, cams, tile, weights)
        out[j] = (Lp - Lm) / (2 * h)
        ok[j] = (sp == sig0) and (sm == sig0)
    return out, ok


# ----------------------------------------------------------------- pruning ----
# The memory-constrained optimisation of Sec. 3.3 (Alg. 1) and the proximal operators of the
# Appendix, written as their plain definitions.

def importance(planes: dict, k: int, cams, tile: int) -> np.ndarray:
    """I_i = sum over the pixels of all views of Gaussian i's blending weight alpha * T
    (Appendix, importance-based selection). Returns float64 [n]."""
    fwd = render(planes, k, cams, tile)
    n = len(planes["op_logit"])
    imp = np.zeros(n * len(cams), np.float64)
    off = fwd["tile_off"]
    for vi, c in enumerate(cams):
        blend(c, tile, fwd["records"], fwd["vals"], fwd["ranges"][off[vi]:off[vi + 1]], importance=imp)
    return imp.reshape(len(cams), n).sum(0)


def topk_keep(score, kappa: int) -> np.ndarray:
    """Mask of the kappa largest scores; equal scores are taken in ascending index order."""
    score = np.asarray(score, np.float64).ravel()
    kappa = max(0, min(int(kappa), score.size))
    order = np.lexsort((np.arange(score.size), -score))
    keep = np.zeros(score.size, bool)
    keep[order[:kappa]] = True
    return keep


def lobe_dynamic_range(z, amp) -> np.ndarray:
    """D = |a| (1 - exp(-2 z)) per lobe (Sec. 3.3.2, the dynamic range of a lobe over the
    sphere), with |a| the Euclidean norm of the RGB amplitude. z [k][n], amp [k][3][n]."""
    a = np.linalg.norm(np.asarray(amp, np.float64), axis=1)
    return a * (1.0 - np.exp(-2.0 * np.asarray(z, np.float64)))


def prox(o, lam_o, imp, kappa_o: int, s, lam_s, amp, kappa_s: int):
    """Proximal step of Alg. 1 with the factorised projection: keep the kappa_o entries of
    o + lambda_o with the highest importance, and the kappa_s lobes of s + lambda_s with the
    highest dynamic range D (evaluated at s + lambda_s); zero the rest."""
    zo = np.asarray(o, np.float64) + np.asarray(lam_o, np.float64)
    zs = np.asarray(s, np.float64) + np.asarray(lam_s, np.float64)
    o_t = np.where(topk_keep(imp, kappa_o), zo, 0.0)
    keep_s = topk_keep(lobe_dynamic_range(zs, amp).ravel(), kappa_s).reshape(zs.shape)
    s_t = np.where(keep_s, zs, 0.0)
    return o_t, s_t


def dual_update(lam, x, x_t):
    """lambda <- lambda + (x - x_tilde) (Alg. 1, dual update)."""
    return np.asarray(lam, np.float64) + (np.asarray(x, np.float64) - np.asarray(x_t, np.float64))


def penalty_grad(grad, delta: float, x, x_t, lam):
    """grad + delta (x - x_tilde + lambda): the augmented-Lagrangian term of the gradient step
    of Alg. 1 (delta_o = delta rho_o, delta_s = delta rho_s)."""
    return np.asarray(grad, np.float64) + delta * (np.asarray(x, np.float64) - np.asarray(x_t, np.float64)
                                                   + np.asarray(lam, np.float64))


# ---------------------------------------------------------- post-processing ----
# Sec. 3.3 (post-processing procedure) and the compensation equation with its derivation in the
# Appendix.

def sphere_mean_factor(s) -> np.ndarray:
    """(1 - e^{-2s}) / (2s): the average of e^{s (mu . d - 1)} over all unit directions d
    (the Appendix's integral, 2 pi (1 - e^{-2s}) / s, over the sphere's area 4 pi); 1 at s = 0."""
    s = np.asarray(s, np.float64)
    out = np.ones_like(s)
    nz = s != 0
    out[nz] = -np.expm1(-2.0 * s[nz]) / (2.0 * s[nz])
    return out


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-np.asarray(x, np.float64)))


def _lobe_table(planes: dict, k: int):
    """Every lobe of the scene as (owner Gaussian, slot, source element), owner-major and slot
    order within a Gaussian, for both lobe layouts."""
    n = len(planes["op_logit"])
    off = planes.get("lobe_off")
    if off is None:
        owner = np.repeat(np.arange(n), k)
        slot = np.tile(np.arange(k), n)
        src = slot * n + owner              # element of sharp[k][n] (flattened)
    else:
        off = np.asarray(off, np.int64)
        cnt = np.diff(off)
        owner = np.repeat(np.arange(n), cnt)
        slot = np.arange(int(off[-1])) - np.repeat(off[:-1], cnt)
        src = np.arange(int(off[-1]))
    return owner, slot, src


def _lobe_values(planes: dict, k: int, src):
    """axis [3][m], sharp [m], amp [3][m], mask [m] of the lobes at source elements src."""
    n = len(planes["op_logit"])
    dense = planes.get("lobe_off") is None
    sh = np.asarray(planes["sharp"], np.float64).reshape(-1)[src]
    if dense:
        slot, owner = src // max(n, 1), src % max(n, 1)
        axis = np.asarray(planes["axis"], np.float64)[slot, :, owner].T
        amp = np.asarray(planes["amp"], np.float64)[slot, :, owner].T
    else:
        axis = np.asarray(planes["axis"], np.float64)[:, src]
        amp = np.asarray(planes["amp"], np.float64)[:, src]
    lm = planes.get("lmask_logit")
    m = np.ones(len(src)) if lm is None else _sigmoid(np.asarray(lm, np.float64).reshape(-1)[src])
    return axis.reshape(3, -1), sh, amp.reshape(3, -1), m


def compact(planes: dict, k: int, opacity_min: float, sharp_min: float) -> dict:
    """Post-processing of Sec. 3.3 on float64 planes (the exact stored values).

    Gaussians with opacity o = sigmoid(op_logit) sigmoid(pmask_logit) below opacity_min are
    removed. Of the rest, lobes with sharpness below sharp_min are removed and each adds its
    compensation m a (1 - e^{-2s}) / (2s) to the base colour (added in slot order); masks are then
    folded (op_logit' = logit(o), amp' = m a), so the result has none. Returns the compacted planes
    in the compressed-row layout with "lobe_off", plus "kept" (source Gaussians) and "lobe_src"
    (source sharpness elements), all float64 except the index arrays."""
    n = len(planes["op_logit"])
    op = np.asarray(planes["op_logit"], np.float64)
    pm = planes.get("pmask_logit")
    o = _sigmoid(op) * (1.0 if pm is None else _sigmoid(pm))
    keep = o >= opacity_min
    kept = np.nonzero(keep)[0]

    owner, slot, src = _lobe_table(planes, k)
    axis, sh, amp, m = _lobe_values(planes, k, src)
    of_kept = keep[owner]
    keep_lobe = of_kept & (sh >= sharp_min)
    drop_lobe = of_kept & ~(sh >= sharp_min)

    base = np.array(planes["base"], np.float64, copy=True)
    comp = m * sphere_mean_factor(np.where(drop_lobe, sh, 0.0))
    for sl in range(max(k, 0)):              # slot order, as the sums are defined
        sel = drop_lobe & (slot == sl)
        for c in range(3):
            np.add.at(base[c], owner[sel], comp[sel] * amp[c, sel])

    if pm is None:
        op_out = op[kept]
    else:
        a, b = op[kept], np.asarray(pm, np.float64)[kept]
        op_out = -np.logaddexp(np.logaddexp(-a, -b), -a - b)   # logit(sigmoid(a) sigmoid(b))

    lsel = np.nonzero(keep_lobe)[0]          # owner-major, slot order: the output order
    cnt = np.bincount(owner[lsel], minlength=n)[kept]
    lobe_off = np.zeros(len(kept) + 1, np.int32)
    lobe_off[1:] = np.cumsum(cnt)
    g = lambda name: np.asarray(planes[name], np.float64)
    return {
        "pos": g("pos")[:, kept], "logscale": g("logscale")[:, kept], "quat": g("quat")[:, kept],
        "op_logit": op_out, "pmask_logit": None, "base": base[:, kept],
        "axis": axis[:, lsel], "sharp": sh[lsel], "amp": amp[:, lsel] * m[lsel], "lmask_logit": None,
        "lobe_off": lobe_off, "kept": kept.astype(np.int32), "lobe_src": src[lsel].astype(np.int32),
    }


# ------------------------------------------------------------ training step ----
# The photometric loss and optimiser of the 3DGS training the paper keeps (Appendix, experimental
# details: the same hyperparameters and optimiser as vanilla 3DGS): L = (1 - lambda) L1 +
# lambda (1 - SSIM), lambda = 0.2, SSIM with an 11x11 Gaussian window of sigma 1.5, zero padding,
# C1 = 0.01^2, C2 = 0.03^2; Adam.

SSIM_C1, SSIM_C2 = 0.01 ** 2, 0.03 ** 2


def gaussian_window(size: int = 11, sigma: float = 1.5) -> np.ndarray:
    """Normalised 1D Gaussian taps; the 2D window is their outer product."""
    x = np.arange(size, dtype=np.float64) - size // 2
    g = np.exp(-x * x / (2.0 * sigma * sigma))
    return g / g.sum()


def photometric_loss(images, targets, lam: float = 0.2):
    """Sum over views of (1 - lam) mean|x - y| + lam (1 - mean SSIM(x, y)) over each view's three
    channels and pixels, and its gradient with respect to every x, in FP64 (plain torch CPU ops
    with autograd; |.| has gradient 0 at x = y). images, targets: lists of [3][H][W] arrays.
    Returns (loss, [dL/dx per view])."""
    import torch
    import torch.nn.functional as F
    g = torch.from_numpy(gaussian_window())
    win = torch.outer(g, g)[None, None]
    total = torch.zeros((), dtype=torch.float64)
    xs = []
    for img, tgt in zip(images, targets):
        x = torch.tensor(np.asarray(img, np.float64), requires_grad=True)
        y = torch.from_numpy(np.asarray(tgt, np.float64))
        xs.append(x)
        conv = lambda t: F.conv2d(t[:, None], win, padding=5)[:, 0]
        mx, my = conv(x), conv(y)
        sxx = conv(x * x) - mx * mx
        syy = conv(y * y) - my * my
        sxy = conv(x * y) - mx * my
        ssim = ((2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2)) / ((mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2))
        total = total + (1 - lam) * (x - y).abs().mean() + lam * (1 - ssim.mean())
    total.backward()
    return float(total.detach()), [x.grad.numpy().copy() for x in xs]


def ssim_map_direct(x, y) -> np.ndarray:
    """The SSIM map of one channel by explicit window sums over zero-padded images (slow; for
    small test images only)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    h, w = x.shape
    g = gaussian_window()
    W = np.outer(g, g)
    xp = np.zeros((h + 10, w + 10)); xp[5:5 + h, 5:5 + w] = x
    yp = np.zeros((h + 10, w + 10)); yp[5:5 + h, 5:5 + w] = y
    out = np.zeros((h, w))
    for i in range(h):
        for j in range(w):
            a = xp[i:i + 11, j:j + 11]
            b = yp[i:i + 11, j:j + 11]
            mx, my = (W * a).sum(), (W * b).sum()
            vx = (W * a * a).sum() - mx * mx
            vy = (W * b * b).sum() - my * my
            cxy = (W * a * b).sum() - mx * my
            out[i, j] = ((2 * mx * my + SSIM_C1) * (2 * cxy + SSIM_C2)) / ((mx * mx + my * my + SSIM_C1) * (vx + vy + SSIM_C2))
    return out


def adam_step(param, grad, m, v, lr: float, beta1: float, beta2: float, eps: float, step: int):
    """One Adam update (Kingma and Ba, with bias correction; eps added to the corrected root):
    returns (param', m', v') in FP64."""
    g = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    return np.asarray(param, np.float64) - lr * mhat / (np.sqrt(vhat) + eps), m, v

"""Helpers for the GPU parity tests: run the HIP path through the C ABI and pull every stage's
buffers back to numpy; compare against the FP64 oracle under the tolerances of the tests."""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from oracle import oracle as O
from paper_2509_07021_amd import _lib as L
from paper_2509_07021_amd import render as R
from paper_2509_07021_amd import scenes as S

IMG_TOL = 1e-5          # max abs image difference (FP32 path vs FP64 oracle)
GRAD_REL = 1e-4         # per-tensor relative L2 and per-element relative tolerance
KEY_BAND = 1e-9         # relative band of the tile level within which either listing decision is accepted


def log(*a):
    print(*a, flush=True)


def flat_weights(weights) -> torch.Tensor:
    return torch.from_numpy(np.concatenate([w.reshape(-1) for w in weights]).astype(np.float32)).cuda()


def gpu_run(scene: S.Scene, cams, cfg: R.Config, weights=None) -> dict:
    """Forward (and backward when weights are given) through the C ABI; all stage buffers as numpy.
    The per-field record planes are requested (MEGS_FLAG_RECORD_PLANES), which only adds their writes."""
    cfg = dataclasses.replace(cfg, flags=cfg.flags | L.MEGS_FLAG_RECORD_PLANES)
    ds = R.DeviceScene.from_scene(scene)
    fr = R.forward(ds, cams, cfg)
    torch.cuda.synchronize()
    st = fr.state
    nr = scene.n * len(cams)
    P = int(st.n_pairs)
    T = int(st.n_tiles)
    npix = int(st.n_pixels)
    out = {"frame": fr, "dscene": ds, "n_pairs": P, "counts": fr.counts()}
    out["images"] = [x.cpu().numpy().astype(np.float64) for x in R.split_images(fr.images, cams)]
    if nr:
        out["mean"] = fr.buffer("mean", 2 * nr, torch.float64).view(nr, 2).cpu().numpy()
        out["conic_o"] = fr.buffer("conic_o", 4 * nr, torch.float32).view(nr, 4).cpu().numpy()
        out["rgbd"] = fr.buffer("rgbd", 4 * nr, torch.float32).view(nr, 4).cpu().numpy()
        out["radius"] = fr.buffer("radius", nr, torch.int32).cpu().numpy()
        out["ntiles"] = fr.buffer("ntiles", nr, torch.int32).cpu().numpy().view(np.uint32)
        out["cutoff"] = fr.buffer("cutoff", nr, torch.float32).cpu().numpy()
        out["chol"] = fr.buffer("chol", 4 * nr, torch.float64).view(nr, 4).cpu().numpy()
    if P:
        out["vals"] = fr.buffer("vals", P, torch.int32).cpu().numpy().view(np.uint32)
        if st.tile_keys:
            out["tile_keys"] = fr.buffer("tile_keys", P, torch.int32).cpu().numpy().view(np.uint32)
        if st.keys64:
            out["keys64"] = fr.buffer("keys64", P, torch.int64).cpu().numpy().view(np.uint64)
    else:
        out["vals"] = np.zeros(0, np.uint32)
    out["ranges"] = fr.buffer("ranges", 2 * T, torch.int32).view(T, 2).cpu().numpy().view(np.uint32)
    out["T_final"] = fr.buffer("T_final", npix, torch.float32).cpu().numpy()
    out["last"] = fr.buffer("last", npix, torch.int32).cpu().numpy().view(np.uint32)
    if weights is not None:
        nblocks = len(fr.alloc.blocks)
        grads = R.backward(ds, fr, flat_weights(weights))
        torch.cuda.synchronize()
        out["grads"] = {p: (None if g is None else g.cpu().numpy().astype(np.float64)) for p, g in grads.items()}
        moments = backward_sums(fr.alloc, fr.state, nblocks, nr)
        out["grad2d_moments"] = moments
        nr0 = out["conic_o"] if nr else np.zeros((0, 4))
        out["grad2d"] = grad2d_from_moments(moments, out["chol"] if nr else np.zeros((0, 4)),
                                            nr0[:, 3].astype(np.float64))
    return out


def grad2d_buffer(block: torch.Tensor, nr: int) -> np.ndarray:
    """The backward's per-record sums [nr][9] from the start of its scratch block (FP64 copy)."""
    return block[: nr * 9 * 4].view(torch.float32).view(nr, 9).cpu().numpy().astype(np.float64)


def backward_sums(alloc, state, nblocks: int, nr: int) -> np.ndarray:
    """The backward's per-record sums: at the start of its scratch, which is the forward's work space
    when that was large enough (no new block), else the first block allocated after the nblocks the
    forward took."""
    if len(alloc.blocks) > nblocks:
        return grad2d_buffer(alloc.blocks[nblocks], nr)
    assert state.work and state.work_bytes >= 36 * nr
    return alloc.view(state.work, 9 * max(nr, 1), torch.float32)[: 9 * nr].view(nr, 9).cpu().numpy().astype(
        np.float64)


# The blend's exponent scale: its exponent in log2 units is -(w1^2 + w2^2), w = KQ2 (l11 (dx + r dy), l22 dy),
# KQ2 = sqrt(log2(e) / 2) rounded to FP32 as the library holds it.
KQ2 = float(np.float32(np.sqrt(np.log2(np.e) / 2)))


def chol_conic(chol: np.ndarray) -> np.ndarray:
    """The conic (a, b, c) that a record's factors (l11, r, l22) describe, in FP64:
    a = l11^2, b = l11^2 r, c = (l11 r)^2 + l22^2."""
    l11, r, l22 = chol[:, 0], chol[:, 1], chol[:, 2]
    a = l11 * l11
    return np.stack([a, a * r, (l11 * r) ** 2 + l22 * l22], axis=1)


def grad2d_from_moments(m: np.ndarray, chol: np.ndarray, oe: np.ndarray) -> np.ndarray:
    """The library's per-record backward buffer holds, per record, the sums over its fragments of
    e w1, e w2, e w1^2, e w1 w2, e w2^2 and e, with e the loss gradient of the effective opacity of an
    unclamped fragment and w = KQ2 (l11 (dx + r dy), l22 dy) the exponent's factors of the pixel
    offset, then the RGB gradients. Back to pixel offsets (dy = w2 / (KQ2 l22), dx = w1 / (KQ2 l11) -
    r dy); the gradient of the Gaussian's exponent q = -(a dx^2 + 2 b dx dy + c dy^2) / 2 is o_eff e.
    Returns the gradients of (u, v, a, b, c, o, r, g, b) that the oracle's blend backward produces,
    for the conic the factors describe. chol: the records' (l11, r, l22, 0); oe: o_eff."""
    g = np.array(m, dtype=np.float64, copy=True)
    l11, r, l22 = chol[:, 0], chol[:, 1], chol[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        i1 = np.where(l11 > 0, 1.0 / (KQ2 * l11), 0.0)
        i2 = np.where(l22 > 0, 1.0 / (KQ2 * l22), 0.0)
    ey = m[:, 1] * i2
    ex = m[:, 0] * i1 - r * ey
    eyy = m[:, 4] * i2 * i2
    pxy = m[:, 3] * i1 * i2
    exy = pxy - r * eyy
    exx = m[:, 2] * i1 * i1 - 2.0 * r * pxy + r * r * eyy
    a, b, c = chol_conic(chol).T
    g[:, 0] = oe * (a * ex + b * ey)
    g[:, 1] = oe * (b * ex + c * ey)
    g[:, 2] = -0.5 * oe * exx
    g[:, 3] = -oe * exy
    g[:, 4] = -0.5 * oe * eyy
    return g


def gpu_records(g: dict) -> dict:
    """The GPU's records in the oracle's record layout (float64 copies of the stored values; the conic
    is the one the stored factors describe, formed in FP64)."""
    m, co, cd = g["mean"], g["conic_o"], g["rgbd"]
    return {"u": m[:, 0].copy(), "v": m[:, 1].copy(), "depth": cd[:, 3].astype(np.float64),
            "conic": chol_conic(g["chol"]), "o": co[:, 3].astype(np.float64),
            "rgb": cd[:, :3].astype(np.float64), "valid": (g["radius"] >= 0).astype(np.int32),
            "radius": g["radius"].astype(np.int32), "cutoff": g["cutoff"].astype(np.float64)}


def check_records(g: dict, rec: dict) -> None:
    """Records against the oracle's (g: the GPU's record planes, rec: the oracle's records, same rows).
    The conic is formed in FP64 and kept as FP32 diagonal factors and an FP64 ratio (the record's
    chol plane, conic = L L'), so it is accurate whatever its condition number: the factors are
    checked against the Cholesky factors of the oracle's FP64 conic, and the FP32 conic plane
    against that conic."""
    valid_o = rec["valid"].astype(bool)
    valid_g = g["radius"] >= 0
    assert np.array_equal(valid_o, valid_g), f"{np.sum(valid_o != valid_g)} culling decisions differ"
    if "counts" in g:   # the library's culled count: the records the oracle finds invalid
        assert g["counts"]["culled"] == int((~valid_o).sum()), (g["counts"], int((~valid_o).sum()))
        assert not g["counts"]["overflow"] and g["counts"]["pairs_needed"] == g["n_pairs"]
    v = valid_g
    np.testing.assert_allclose(g["mean"][v, 0], rec["u"][v], rtol=0, atol=1e-9)
    np.testing.assert_allclose(g["mean"][v, 1], rec["v"][v], rtol=0, atol=1e-9)
    np.testing.assert_allclose(g["rgbd"][v, 3], rec["depth"][v], rtol=1e-6)
    np.testing.assert_allclose(g["conic_o"][v, :3], rec["conic"][v], rtol=2e-5,
                               atol=2e-5 * np.abs(rec["conic"][v]).max())
    # the factors: l11 = sqrt(a), r = b / a, l22 = sqrt(c - b^2 / a) of the oracle's conic (a, b, c)
    oc = rec["conic"][v]
    l11 = np.sqrt(oc[:, 0])
    ratio = oc[:, 1] / oc[:, 0]
    l22 = np.sqrt((oc[:, 0] * oc[:, 2] - oc[:, 1] ** 2) / oc[:, 0])
    ch = g["chol"][v]
    np.testing.assert_allclose(ch[:, 0], l11, rtol=2e-6)
    np.testing.assert_allclose(ch[:, 2], l22, rtol=2e-6)
    # the ratio carries the footprint's direction: relative to the factors' own precision it is exact
    rerr = np.abs(ch[:, 1] - ratio) / (1.0 + np.abs(ratio))
    assert rerr.max() <= 2e-6, f"factor ratio error {rerr.max():.2e}"
    np.testing.assert_allclose(g["conic_o"][v, 3], rec["o"][v], rtol=2e-6)
    np.testing.assert_allclose(g["rgbd"][v, :3], rec["rgb"][v], rtol=0, atol=2e-6)
    dr = np.abs(g["radius"][v] - rec["radius"][v])
    assert dr.max() <= 1 and (dr > 0).mean() < 1e-3
    np.testing.assert_allclose(g["cutoff"][v], rec["cutoff"][v], rtol=1e-5, atol=1e-5)


def view_pixels(cams, vi):
    off = sum(c.width * c.height for c in cams[:vi])
    return off, cams[vi].width * cams[vi].height


def grad_close(name, g, ref, rel=GRAD_REL, abs_sum=None):
    """Gradient parity.

    Per tensor: ||g - ref||_2 / ||ref||_2 <= rel (the stated 1e-4 relative tolerance).
    Per element, as a guard against localised errors: when abs_sum (the oracle's sum of the
    absolute values of the contributions summed into each element) is given,
    |g - ref| <= rel * (|ref| + abs_sum) + 1e-3 * rel * max|ref|; otherwise
    |g - ref| <= rel * |ref| + 1e-2 * rel * max|ref|. Summing FP32 terms in any order errs
    relative to the terms' absolute sum, not to their (possibly cancelling) total, which is what
    both forms allow for; the small floor covers terms that cancel inside themselves (a colour
    minus the background accumulated behind it, a transmittance recovered through hundreds of
    divisions), which matters only for elements some 1e-7 of the tensor's largest.
    """
    assert g.shape == ref.shape, (name, g.shape, ref.shape)
    g, ref = np.ravel(g), np.ravel(ref)
    if abs_sum is not None:
        abs_sum = np.ravel(abs_sum)
    if ref.size == 0:
        return 0.0
    scale = np.abs(ref).max()
    if scale == 0:
        assert np.abs(g).max() == 0, name
        return 0.0
    d = np.abs(g - ref)
    l2 = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    assert l2 <= rel, f"{name}: relative L2 {l2:.3e}"
    if abs_sum is not None:
        bound = rel * (np.abs(ref) + abs_sum) + 1e-3 * rel * scale
    else:
        bound = rel * np.abs(ref) + 1e-2 * rel * scale
    bad = d > bound
    ratio = np.divide(d, bound, out=np.zeros_like(d), where=bound > 0)
    i = int(np.argmax(np.where(bad, np.inf, ratio)))
    assert not bad.any(), (f"{name}: {bad.sum()} elements over; worst {ratio.max():.2f}x at {i}: "
                           f"got {g[i]:.6e}, oracle {ref[i]:.6e}")
    return l2


def scene_from_device(ds: R.DeviceScene) -> S.Scene:
    """A DeviceScene's planes back on the host as a scenes.Scene (bf16 as uint16 bit patterns)."""
    def host(t):
        if t is None:
            return None
        t = t.detach().cpu()
        if t.dtype == torch.bfloat16:
            return t.view(torch.int16).numpy().view(np.uint16).copy()
        return t.numpy().copy()
    planes = {p: host(ds.planes.get(p)) for p in S.PLANES}
    lobe_off = None if ds.lobe_off is None else ds.lobe_off.cpu().numpy().astype(np.int32)
    return S.Scene(n=ds.n, k=ds.k, dt_geom=ds.dt[0], dt_color=ds.dt[1], dt_amp=ds.dt[2], lobe_off=lobe_off,
                   **planes)


def check_key_table(vals, ranges, rec, depth_f32, cams, tile: int, n: int, tile_keys=None, keys64=None,
                    sub: int = 0) -> dict:
    """The GPU's key table against the oracle's plain tile definition, given the same records.

    The oracle lists a (tile, record) pair when the minimum of the record's quadratic form over the
    tile's pixel-centre box is at most the record's level k. Pairs whose minimum lies within KEY_BAND k
    of k are flagged: the kernel evaluates the same definition in another FP64 rounding order and may
    take either side, so there the GPU's decision is adopted, and the flagged pairs are counted. Every
    other decision, and then the sorted keys, record order and per-tile ranges, must agree bit for bit.
    With sub-tile flags (sub = 8), the upper 16 bits of each tile key must flag every 8 x 8 sub-tile the
    ellipse reaches (the flags are a superset: the kernel widens them); the extra flags are counted.
    Returns the counts."""
    nv = len(cams)
    rec_view = np.repeat(np.arange(nv, dtype=np.int32), n)
    tl, rc, st = O.tile_candidates(rec["u"], rec["v"], rec["radius"], rec["conic"], rec["cutoff"], rec["valid"],
                                   rec_view, cams, tile, KEY_BAND)
    off = O.tile_layout(cams, tile)
    vals = np.asarray(vals, np.uint32)
    if keys64 is not None:
        gtile = (np.asarray(keys64, np.uint64) >> np.uint64(32)).astype(np.int64)
    else:
        tk = np.asarray(tile_keys, np.uint32)
        gtile = (tk & np.uint32(0xFFFF) if sub else tk).astype(np.int64)
    near = st == 2
    gcode = (gtile << 32) | vals.astype(np.int64)
    ncode = (tl[near] << 32) | rc[near].astype(np.int64)
    taken = np.isin(ncode, gcode)
    keep = st == 1
    keep[np.nonzero(near)[0][taken]] = True
    depth_bits = np.asarray(depth_f32, np.float32).view(np.uint32).astype(np.uint64)
    keys = (tl[keep].astype(np.uint64) << np.uint64(32)) | depth_bits[rc[keep]]
    okeys, ovals, oranges = O.sort_pairs(keys, rc[keep], int(off[-1]))
    assert len(vals) == len(ovals), f"{len(vals)} pairs listed, oracle {len(ovals)} ({int(near.sum())} in the band)"
    np.testing.assert_array_equal(vals, ovals)
    np.testing.assert_array_equal(np.asarray(ranges, np.uint32).reshape(-1, 2), oranges)
    np.testing.assert_array_equal(gtile.astype(np.uint64), okeys >> np.uint64(32))
    if keys64 is not None:
        np.testing.assert_array_equal(np.asarray(keys64, np.uint64), okeys)
    out = {"pairs": int(len(vals)), "band": int(near.sum()), "band_listed": int(taken.sum())}
    assert out["band"] <= 1e-5 * max(len(vals), 1) + 2, out
    if sub and tile_keys is not None and len(vals):
        flags = np.asarray(tile_keys, np.uint32) >> np.uint32(16)
        fset, fnear = O.subtile_flags(gtile, vals, rec["u"], rec["v"], rec["conic"], rec["cutoff"], rec_view, cams,
                                      tile, KEY_BAND)
        missing = fset & ~flags
        assert not missing.any(), f"{np.count_nonzero(missing)} pairs miss the flag of a reached sub-tile"
        pc = lambda x: int(np.unpackbits(x.view(np.uint8)).sum())
        out["subtiles"] = pc(fset)
        out["subtiles_extra"] = pc(flags & ~fset & ~fnear)
    return out

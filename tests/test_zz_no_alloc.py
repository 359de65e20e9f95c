"""The forward that allocates nothing (megs_render_forward_noalloc, for callers that cannot allocate)
against megs_render_forward, through the C ABI: two calls in a row on one device, the second on a
smaller input, each compared with the allocating forward on the same input. Both run the same
kernels, so images, transmittance, last indices, the key table and the ranges must agree bit for
bit; the state the no-allocation call leaves must also feed the ordinary backward."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2509_07021_amd import _lib as L
from paper_2509_07021_amd import render as R
from paper_2509_07021_amd import scenes as S

pytestmark = pytest.mark.gpu

_HIP = None


def _d2h(ptr: int, count: int, dtype) -> np.ndarray:
    """Copies count elements at a device address into a numpy array (synchronous hipMemcpy)."""
    global _HIP
    if _HIP is None:
        _HIP = ctypes.CDLL("libamdhip64.so")
        _HIP.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _HIP.hipMemcpy.restype = ctypes.c_int
    out = np.empty(count, dtype)
    if count:
        assert ptr, "null device pointer"
        rc = _HIP.hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2)  # hipMemcpyDeviceToHost
        assert rc == 0, f"hipMemcpy failed with {rc}"
    return out


def _noalloc(ds, cams, cfg):
    lib = L.load()
    npix = sum(c.width * c.height for c in cams)
    images = torch.full((3 * npix,), float("nan"), dtype=torch.float32, device="cuda")
    st = L.MegsState()
    sc, cam_arr, c = ds.struct(), R.cameras_struct(cams), cfg.struct()
    torch.cuda.synchronize()
    L.check(lib.megs_render_forward_noalloc(ctypes.byref(sc), cam_arr, len(cams), ctypes.byref(c),
                                            images.data_ptr(), ctypes.byref(st), R._stream(None)))
    torch.cuda.synchronize()
    return images, st


def _outputs(state, images):
    lib = L.load()
    counted = ctypes.c_int64()
    L.check(lib.megs_state_status(ctypes.byref(state), ctypes.byref(counted), R._stream(None)))
    P, T, npix = int(counted.value), int(state.n_tiles), int(state.n_pixels)
    assert P <= int(state.pair_capacity)
    return {"images": images.cpu().numpy(), "T_final": _d2h(state.T_final, npix, np.float32),
            "last": _d2h(state.last, npix, np.uint32), "vals": _d2h(state.vals, P, np.uint32),
            "tile_keys": _d2h(state.tile_keys, P, np.uint32) if state.tile_keys else None,
            "ranges": _d2h(state.ranges, 2 * T, np.uint32), "n_pairs": P}


def _case(scene, cams, cfg, label):
    print(f"no-alloc case {label}: n={scene.n}, {cams[0].width}x{cams[0].height} x{len(cams)}, "
          f"tile={cfg.tile}, subtile={cfg.subtile}, capacity={cfg.pair_capacity}", flush=True)
    ds = R.DeviceScene.from_scene(scene)
    ref = R.forward(ds, cams, cfg)
    torch.cuda.synchronize()
    want = _outputs(ref.state, ref.images)
    images, st = _noalloc(ds, cams, cfg)
    got = _outputs(st, images)
    assert got["n_pairs"] == want["n_pairs"] > 0
    for key in ("images", "T_final", "last", "vals", "tile_keys", "ranges"):
        if want[key] is None:
            assert got[key] is None, key
            continue
        np.testing.assert_array_equal(got[key], want[key], err_msg=key)
    assert np.isfinite(got["images"]).all()
    # the no-allocation state feeds the ordinary backward: the same gradients as the allocating path
    # (float atomics add in another order, so within FP32 rounding of the summed terms)
    dl = torch.from_numpy(np.concatenate([x.reshape(-1) for x in S.loss_weights(cams, 7)])).cuda()
    g_ref = R.backward(ds, ref, dl)
    frame = R.Frame(images, st, R.TorchAllocator(), cams, cfg)
    g_got = R.backward(ds, frame, dl)
    torch.cuda.synchronize()
    for p, t in g_ref.items():
        if t is None:
            continue
        a, b = g_got[p].cpu().numpy().astype(np.float64), t.cpu().numpy().astype(np.float64)
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        assert rel <= 1e-5, (p, rel)


@pytest.mark.parametrize("capacity", [0, 300_000])
def test_noalloc_forward_matches_forward_twice(capacity):
    scene, cams = S.make_workload("small_2k_128px")
    cfg = R.Config(32, 64, subtile=8, pair_capacity=capacity)
    _case(scene, cams, cfg, "first")
    # second call on the same device: a smaller input (fewer Gaussians, a smaller image, 16x16 tiles);
    # the array still holds the first call's contents
    small = scene.subset(np.arange(0, scene.n, 3))
    cam = S.crop_camera(cams[0], 96, 80)
    _case(small, [cam], R.Config(16, 64, pair_capacity=capacity // 2), "second")


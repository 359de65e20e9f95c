"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle, stage by stage and end
to end. Tolerances: images 1e-5 max abs; gradients 1e-4 relative per tensor (L2), with a
per-element guard scaled by each element's absolute contribution sum (see gpu_util.grad_close);
keys, order and ranges bit-exact given the same record means, depths and radii. Pixels whose oracle decisions lie within the threshold
bands are excluded from image comparisons and get zero loss weight in gradient comparisons.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_07021_amd import render as R
from paper_2509_07021_amd import scenes as S

from gpu_util import IMG_TOL, check_key_table, check_records, grad_close, gpu_records, gpu_run, log, view_pixels

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - the marker keeps these off CPU runs
    pytest.skip("no GPU", allow_module_level=True)


def _oracle_masked_weights(scene, cams, tile, seed):
    """Loss weights with zeros on pixels the oracle flags as near a decision threshold."""
    fwd = O.render(scene.widened(), scene.k, cams, tile)
    w = S.loss_weights(cams, seed)
    wm = [wi * (1 - vw["flag"])[None].astype(np.float32) for wi, vw in zip(w, fwd["views"])]
    return fwd, wm


def conic_condition(conic):
    """Condition number lambda_max / lambda_min of each 2x2 conic (a, b, c)."""
    tr, det = conic[:, 0] + conic[:, 2], conic[:, 0] * conic[:, 2] - conic[:, 1] ** 2
    lam = tr / 2 + np.sqrt(np.maximum(tr * tr / 4 - det, 0))
    return lam * lam / det


def _check_records(g, fwd, n_views):
    check_records(g, fwd["records"])


def _check_key_stage(g, cams, tile, n, sub=0):
    """Keys, order and ranges from the GPU's own records against the oracle's plain tile definition
    (gpu_util.check_key_table): bit-exact outside the flagged band; with sub-tile blending, the tile
    keys' upper 16 bits flag every sub-tile the ellipse reaches."""
    rec = gpu_records(g)
    if g["n_pairs"]:
        cnt = check_key_table(g["vals"], g["ranges"], rec, g["rgbd"][:, 3], cams, tile, n,
                              tile_keys=g.get("tile_keys"), keys64=g.get("keys64"), sub=sub)
        log(f"key table: {cnt}")
    else:
        assert not g["ranges"].any()
    return rec, O.tile_layout(cams, tile)


def _check_blend_stage(g, rec, cams, tile, off, img_tol=IMG_TOL, t_rtol=1e-5):
    """The blend over the GPU's own records and lists against the oracle's compositor: last
    indices (every alpha and termination decision) exactly, colour and transmittance within the
    given tolerances."""
    worst = 0.0
    for vi, cam in enumerate(cams):
        ob = O.blend(cam, tile, rec, g["vals"], g["ranges"][off[vi]:off[vi + 1]])
        ok = ob["flag"] == 0
        d = np.abs(g["images"][vi] - ob["image"])[:, ok]
        worst = max(worst, float(d.max()) if d.size else 0.0)
        p0, npx = view_pixels(cams, vi)
        last = g["last"][p0:p0 + npx].reshape(cam.height, cam.width)
        assert np.array_equal(last[ok], ob["last"][ok])
        T = g["T_final"][p0:p0 + npx].reshape(cam.height, cam.width)
        np.testing.assert_allclose(T[ok], ob["T"][ok], rtol=t_rtol, atol=1e-7)
    assert worst <= img_tol, worst
    return worst


def _run_all_stages(scene, cams, cfg, seed=7):
    """Every stage against the oracle: stage-wise on the GPU's own records (keys, order, ranges and
    last indices bit-exact, blend and blend backward within the FP32 tolerances), then end to end
    against the FP64 pipeline. Returns the GPU's buffers, the oracle's forward and the measured
    end-to-end errors (max abs image error; per-tensor relative gradient errors)."""
    log(f"case n={scene.n} k={scene.k} views={len(cams)} tile={cfg.tile} batch={cfg.batch} flags={cfg.flags}")
    fwd, w = _oracle_masked_weights(scene, cams, cfg.tile, seed)
    g = gpu_run(scene, cams, cfg, weights=w)
    _check_records(g, fwd, len(cams))
    rec, off = _check_key_stage(g, cams, cfg.tile, scene.n, sub=cfg.subtile)
    _check_blend_stage(g, rec, cams, cfg.tile, off)
    # end-to-end images against the FP64 pipeline
    e2e = {"image": 0.0}
    for vi in range(len(cams)):
        ok = fwd["views"][vi]["flag"] == 0
        d = np.abs(g["images"][vi] - fwd["images"][vi])[:, ok]
        e2e["image"] = max(e2e["image"], float(d.max()))
        assert d.max() <= IMG_TOL, (vi, d.max())
    # backward, stage-wise: blend backward over the GPU's records and lists
    g2_ref = np.zeros_like(g["grad2d"])
    g2_abs = np.zeros_like(g["grad2d"])
    for vi, cam in enumerate(cams):
        O.blend_backward(cam, cfg.tile, rec, g["vals"], g["ranges"][off[vi]:off[vi + 1]], w[vi], grad2d=g2_ref,
                         grad2d_abs=g2_abs)
    for c, name in enumerate(("u", "v", "a", "b", "c", "o", "r", "g", "b_col")):
        e2e[f"grad2d[{name}]"] = grad_close(f"grad2d[{name}]", g["grad2d"][:, c], g2_ref[:, c], abs_sum=g2_abs[:, c])
    # projection backward, stage-wise: fed with the GPU's 2D gradients
    pl = scene.widened()
    gr_stage = O.zero_grads(pl)
    n = scene.n
    for vi, cam in enumerate(cams):
        O.project_backward(pl, scene.k, cam, cfg.tile, g["grad2d"][vi * n:(vi + 1) * n], gr_stage)
    for p in O.PLANES:
        if gr_stage[p] is not None:
            e2e[f"stage {p}"] = grad_close(f"stage {p}", g["grads"][p], gr_stage[p])
    # end to end against the FP64 gradient
    gr, _ = O.render_backward(pl, scene.k, cams, cfg.tile, w, fwd=fwd)
    for p in O.PLANES:
        if gr[p] is not None:
            e2e[p] = grad_close(p, g["grads"][p], gr[p])
    log("errors: " + ", ".join(f"{k} {v:.2e}" for k, v in e2e.items()))
    return g, fwd, e2e


def test_small_workload_all_stages():
    scene, cams = S.make_workload("small_2k_128px")
    _run_all_stages(scene, cams, R.Config(16, 64))


@pytest.mark.parametrize("tile,batch,waves", [(8, 64, 1), (16, 32, 1), (16, 128, 2), (16, 64, 4), (32, 256, 1),
                                               (32, 64, 2), (32, 128, 4)])
def test_tile_batch_and_wave_variants(tile, batch, waves):
    scene, cams = S.make_workload("small_2k_128px")
    _run_all_stages(scene, cams, R.Config(tile, batch, waves=waves))


@pytest.mark.parametrize("tile", [16, 32])
def test_subtile_blend(tile):
    """One independent wave per 8x8 sub-tile walking the tile's list: every stage against the
    oracle, on views with ragged edges (sub-tiles past the image edge)."""
    scene, cams = S.make_workload("small_2k_128px")
    cams = cams + [S.look_at((2.0, -3.0, 1.5), 100, 60, bg=(0.2, 0.2, 0.2))]
    _run_all_stages(scene, cams, R.Config(tile, 64, subtile=8))


def test_one_stage_sort_matches_two_stage():
    scene, cams = S.make_workload("small_2k_128px")
    cams = cams + [S.look_at((2.0, -3.0, 1.5), 100, 60)]
    a = gpu_run(scene, cams, R.Config(16, 64))
    b = gpu_run(scene, cams, R.Config(16, 64, flags=1))
    np.testing.assert_array_equal(a["vals"], b["vals"])
    np.testing.assert_array_equal(a["ranges"], b["ranges"])
    for x, y in zip(a["images"], b["images"]):
        np.testing.assert_array_equal(x, y)
    _check_key_stage(b, cams, 16, scene.n)


def test_masked_crop_gradients():
    """The masked 1M workload's 500-Gaussian crop (64x64 centre window), mask gradients included."""
    scene, cams = S.make_workload("masked_1m_1080p", n=200_000)
    idx = S.axis_nearest(scene, cams[0], 500)
    crop = scene.subset(idx)
    cam = S.crop_camera(cams[0], 64, 64)
    g, _, _ = _run_all_stages(crop, [cam], R.Config(16, 64), seed=3)
    assert np.abs(g["grads"]["pmask_logit"]).max() > 0 and np.abs(g["grads"]["lmask_logit"]).max() > 0


def test_multiview_uneven_and_ragged():
    rng = np.random.default_rng(5)
    scene = S.random_scene(rng, 3000, 4, masks=True, spread=1.0, logscale_mu=-3.0)
    cams = [S.look_at((0, -4, 0.3), 100, 37), S.look_at((3, -2, 1), 64, 64, bg=(0.2, 0.3, 0.4)),
            S.look_at((-2.5, 2.5, 1.5), 150, 90), S.look_at((0.5, 0.5, 4.0), 33, 129)]
    _run_all_stages(scene, cams, R.Config(16, 64))


def test_reduced_precision_storage():
    """FP16 planes with BF16 amplitudes, widened in registers; oracle reads the exact stored values."""
    scene, cams = S.make_workload("clustered_200k_720p", n=20_000)
    scene = scene.stored("f16", "f16", "bf16")
    cams = [S.crop_camera(cams[0], 320, 180)]
    _run_all_stages(scene, cams, R.Config(16, 64))


def test_bf16_geometry_and_colour_storage():
    """The other storage combination: geometry and colour planes in BF16, amplitudes in FP16 (each
    parameter group is loaded and widened under its own type), in the benchmark's launch
    configuration; the oracle reads the exact stored values."""
    scene, cams = S.make_workload("clustered_200k_720p", n=20_000)
    scene = scene.stored("bf16", "bf16", "f16")
    cams = [S.crop_camera(cams[0], 320, 180)]
    _run_all_stages(scene, cams, R.Config(32, 64, subtile=8), seed=4)


def test_forward_is_deterministic():
    scene, cams = S.make_workload("small_2k_128px")
    a = gpu_run(scene, cams, R.Config(16, 64))
    b = gpu_run(scene, cams, R.Config(16, 64))
    for x, y in zip(a["images"], b["images"]):
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(a["vals"], b["vals"])


def test_empty_and_culled_scenes():
    cams = [S.look_at((0, -4, 0), 40, 24, bg=(0.25, 0.5, 0.75))]
    empty = S.random_scene(np.random.default_rng(0), 0, 2, masks=False)
    g = gpu_run(empty, cams, R.Config(8, 64))
    np.testing.assert_array_equal(g["images"][0], np.broadcast_to(np.array([0.25, 0.5, 0.75])[:, None, None],
                                                                  (3, 24, 40)).astype(np.float32))
    behind = S.random_scene(np.random.default_rng(1), 50, 2, masks=False, spread=0.2)
    behind.pos[1] -= 6.0  # all behind the camera at y = -4
    g = gpu_run(behind, cams, R.Config(8, 64))
    assert g["n_pairs"] == 0 and (g["radius"] < 0).all()
    assert g["counts"]["culled"] == 50 and g["counts"]["pairs_needed"] == 0
    np.testing.assert_array_equal(g["images"][0].astype(np.float32), np.broadcast_to(
        np.array([0.25, 0.5, 0.75], np.float32)[:, None, None], (3, 24, 40)))


@pytest.mark.parametrize("tile,sub", [(32, 8), (16, 0)])
def test_needle_footprints(tile, sub):
    """Needle-shaped Gaussians (one long axis, two very thin ones): 2D conics with condition numbers
    in the thousands, where an FP32 determinant or quadratic form would cancel most and the culling
    box and sub-tile flags of a thin ellipse are tightest; every stage against the oracle at the
    standard tolerances (images 1e-5, gradients 1e-4), in the benchmark's launch configuration
    (32x32 tiles, 8x8 sub-tiles) and a per-tile one. The shape is projected in FP64 and the blend's
    exponent is a sum of squares staged per sub-tile, so nothing here depends on the condition
    number (measured: images 7e-7 max abs, gradients 5e-5 per tensor at most, for the log-scales)."""
    rng = np.random.default_rng(11)
    scene = S.random_scene(rng, 600, 3, masks=True, spread=0.8, logscale_mu=-4.0)
    scene.logscale[0] = rng.uniform(-0.3, 0.7, scene.n).astype(np.float32)
    scene.logscale[1:] = rng.uniform(-7.0, -5.5, (2, scene.n)).astype(np.float32)
    cams = [S.look_at((0, -4, 0.5), 120, 96), S.look_at((3, -2, 1), 72, 72, bg=(0.1, 0.2, 0.3))]
    g, fwd, e2e = _run_all_stages(scene, cams, R.Config(tile, 64, subtile=sub), seed=5)
    rec = fwd["records"]
    assert conic_condition(rec["conic"][rec["valid"].astype(bool)]).max() > 1e3  # thin ellipses reached


@pytest.mark.parametrize("tile,sub,min_pairs", [(8, 0, 16 * 2048), (32, 8, 2 * 2048)])
def test_emission_spans_many_windows(tile, sub, min_pairs):
    """Large footprints (400 Gaussians of tens of pixels radius in one 320x240 view): the key
    emission's two workgroups of up to 256 records each emit several times its LDS window of 2048
    pairs, so records' tile runs straddle window boundaries (about 18 windows per workgroup with 8x8
    tiles, 2-3 with 32x32 tiles and sub-tile flags); keys, order and ranges bit-exact against the
    oracle's plain tile definition, and every later stage at the standard tolerances."""
    scene = S.random_scene(np.random.default_rng(21), 400, 2, masks=True, spread=1.0, logscale_mu=-1.2)
    cams = [S.look_at((0, -4, 0.3), 320, 240, bg=(0.2, 0.1, 0.3))]
    g, _, _ = _run_all_stages(scene, cams, R.Config(tile, 64, subtile=sub), seed=9)
    assert g["n_pairs"] > min_pairs, g["n_pairs"]


def test_misaligned_allocation_is_rejected():
    """The allocation callback must return 256-byte aligned memory: a pointer that is not (here 16
    bytes past an aligned block) fails with MEGS_ERR_ALLOC before anything is launched, and the
    same call with aligned memory still renders."""
    import ctypes
    from paper_2509_07021_amd import _lib as L
    scene, cams = S.make_workload("small_2k_128px")
    ds = R.DeviceScene.from_scene(scene)
    lib = L.load()
    blocks = []

    def make(shift):
        def _alloc(ctx, nbytes):
            t = torch.empty(int(nbytes) + 512, dtype=torch.uint8, device="cuda")
            blocks.append(t)
            base = (t.data_ptr() + 255) // 256 * 256
            return base + shift
        return L.ALLOC_FN(_alloc)

    sc = ds.struct(None)
    cam_arr = R.cameras_struct(cams)
    cfg = R.Config(32, 64, subtile=8).struct()
    images = torch.zeros(3 * 128 * 128, device="cuda")
    for shift, expect in ((16, L.MEGS_ERR_ALLOC), (0, L.MEGS_OK)):
        fn = make(shift)
        state = L.MegsState()
        rc = lib.megs_render_forward(ctypes.byref(sc), cam_arr, len(cams), ctypes.byref(cfg), fn, None,
                                     images.data_ptr(), ctypes.byref(state), R._stream(None))
        torch.cuda.synchronize()
        assert rc == expect, (shift, rc, lib.megs_last_error().decode())
        if shift:
            assert "256-byte aligned" in lib.megs_last_error().decode()
            assert float(images.abs().max()) == 0.0  # nothing was rendered
    assert float(images.abs().max()) > 0.0


def test_pair_count_beyond_32_bits():
    """1200 Gaussians that each cover a whole 16384 x 16384 view reach all of its 2048 x 2048 8x8
    tiles: about 5.0e9 tile pairs, more than 32 bits count. The pair count is summed in 64 bits and
    saturated, so the eager forward refuses the work (MEGS_ERR_CAPACITY) instead of sizing a table
    from a wrapped count; with a fixed capacity the forward runs, flags the overflow and reports
    2^31 - 1 pairs needed (the most a key table holds)."""
    import ctypes
    from paper_2509_07021_amd import _lib as L
    rng = np.random.default_rng(21)
    scene = S.random_scene(rng, 1200, 0, masks=False, spread=0.2)
    scene.logscale[:] = 0.7
    scene.op_logit[:] = 4.0
    cams = [S.look_at((0, -4, 0), 16384, 16384)]
    ds = R.DeviceScene.from_scene(scene)
    log("pair count beyond 32 bits: eager forward")
    with pytest.raises(L.MegsError) as e:
        R.forward(ds, cams, R.Config(8, 64))
    assert e.value.status == L.MEGS_ERR_CAPACITY and "at least 4294967295" in str(e.value), str(e.value)
    log("pair count beyond 32 bits: fixed capacity")
    fr = R.forward(ds, cams, R.Config(8, 64, L.MEGS_FLAG_RECORD_PLANES, pair_capacity=1 << 16))
    c = fr.counts()
    assert c["overflow"] and c["pairs_needed"] == (1 << 31) - 1 and c["culled"] == 0, c
    need = ctypes.c_int64(0)
    rc = L.load().megs_state_status(ctypes.byref(fr.state), ctypes.byref(need), R._stream(None))
    assert rc == L.MEGS_ERR_CAPACITY and need.value == (1 << 31) - 1
    nt = fr.alloc.view(fr.state.ntiles, scene.n, torch.int32).cpu().numpy()
    assert (nt == 2048 * 2048).all()   # every record reaches every tile


@pytest.mark.parametrize("tile,sub,flags", [(16, 0, 0), (32, 8, 0), (8, 0, 1), (16, 0, 8)])
def test_state_bytes_match_the_allocations(tile, sub, flags):
    """megs_state_bytes predicts the blocks the forward and the backward ask for (eager, then as one
    graph with a fixed capacity), and a backward that takes the forward's work space allocates nothing
    and computes the same gradients as one with memory of its own (the deterministic mode's)."""
    import ctypes
    from paper_2509_07021_amd import _lib as L
    scene, cams = S.make_workload("small_2k_128px")
    ds = R.DeviceScene.from_scene(scene)
    cfg = R.Config(tile, 64, flags, subtile=sub)
    lib = L.load()

    def predicted(c, n_pairs):
        m = L.MegsMemory()
        L.check(lib.megs_state_bytes(ctypes.byref(ds.struct()), R.cameras_struct(cams), len(cams),
                                     ctypes.byref(c.struct()), n_pairs, ctypes.byref(m)))
        return m

    fr = R.forward(ds, cams, cfg)
    P = int(fr.state.n_pairs)
    m = predicted(cfg, P)
    sizes = [b.numel() for b in fr.alloc.blocks]
    assert sizes == [m.frame, m.pairs], (sizes, m.frame, m.pairs)
    npix = sum(c.width * c.height for c in cams)
    dl = torch.from_numpy(np.concatenate([w.reshape(-1) for w in S.loss_weights(cams, 4)])).cuda()
    grads = R.backward(ds, fr, dl)
    torch.cuda.synchronize()
    sizes = [b.numel() for b in fr.alloc.blocks]
    assert sizes == [m.frame, m.pairs] + ([m.backward] if m.backward else []), (sizes, m.backward)
    log(f"tile {tile} sub {sub} flags {flags}: frame {m.frame} (work {m.work}), pairs {m.pairs}, "
        f"backward {m.backward}")
    if not flags & L.MEGS_FLAG_DETERMINISTIC:
        assert m.backward == 0 and fr.state.work
    fixed = dataclasses.replace(cfg, pair_capacity=P + 100)
    G = R.Graph(ds, cams, fixed, with_backward=True, dl_images=dl)
    G.launch()
    G.stream.synchronize()
    mg = predicted(fixed, 0)
    sizes = [b.numel() for b in G.alloc.blocks]
    assert sizes == [mg.frame, mg.pairs] + ([mg.backward] if mg.backward else []), (sizes, mg.frame, mg.pairs)
    for p, g in grads.items():   # the same sums (bit for bit in the deterministic mode)
        if g is not None:
            ref, got = g.cpu().numpy(), G.grads[p].cpu().numpy()
            if flags & L.MEGS_FLAG_DETERMINISTIC:
                np.testing.assert_array_equal(got, ref)
            else:
                assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref), p
    G.close()


def test_zero_lobes_and_single_gaussian():
    rng = np.random.default_rng(9)
    scene = S.random_scene(rng, 1, 0, masks=False, spread=0.1, logscale_mu=-1.5)
    _run_all_stages(scene, [S.look_at((0, -3, 0), 48, 40)], R.Config(16, 64))


@pytest.mark.parametrize("tile,waves,flags,sub", [(16, 4, 8, 0), (8, 1, 8, 0), (32, 2, 8 | 2, 0), (16, 1, 8 | 1, 0),
                                                  (16, 1, 8, 8)])
def test_deterministic_backward_is_bitwise_reproducible(tile, waves, flags, sub):
    """MEGS_FLAG_DETERMINISTIC: per-pair gradient slots summed per record in a fixed order. Every
    stage still matches the oracle, and two runs give bit-identical gradients (with sub-tile
    blending the forward runs per sub-tile and the backward per tile)."""
    scene, cams = S.make_workload("small_2k_128px")
    cams = cams + [S.look_at((2.0, -3.0, 1.5), 100, 60, bg=(0.2, 0.2, 0.2))]
    cfg = R.Config(tile, 64, flags=flags, waves=waves, subtile=sub)
    g1, fwd, _ = _run_all_stages(scene, cams, cfg)
    w = [np.asarray(x) for x in S.loss_weights(cams, 7)]
    g2 = gpu_run(scene, cams, cfg, weights=[wi * (1 - vw["flag"])[None].astype(np.float32)
                                            for wi, vw in zip(w, fwd["views"])])
    np.testing.assert_array_equal(g1["grad2d"], g2["grad2d"])
    for p, a in g1["grads"].items():
        if a is not None:
            np.testing.assert_array_equal(a, g2["grads"][p])

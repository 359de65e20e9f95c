"""GPU tests of the batched form (hipGraph capture and replay, persistent work queue, autotuner,
capacity overflow) and of the full-size workloads on sampled outputs."""
import ctypes
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_07021_amd import _lib as L
from paper_2509_07021_amd import render as R
from paper_2509_07021_amd import scenes as S

from gpu_util import (IMG_TOL, backward_sums, check_key_table, check_records, grad2d_from_moments, grad_close,
                      gpu_records, gpu_run, log)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)


def _uneven():
    rng = np.random.default_rng(17)
    scene = S.random_scene(rng, 6000, 4, masks=True, spread=1.2, logscale_mu=-3.2)
    cams = [S.look_at((0, -4, 0.3), 160, 90), S.look_at((3, -2, 1), 96, 96, bg=(0.2, 0.3, 0.4)),
            S.look_at((-2.5, 2.5, 1.5), 200, 120), S.look_at((0.5, 0.5, 4.0), 48, 136)]
    return scene, cams


def _eager(ds, cams, cfg, dl):
    fr = R.forward(ds, cams, cfg)
    grads = R.backward(ds, fr, dl)
    torch.cuda.synchronize()
    return fr, {p: (None if g is None else g.cpu().numpy()) for p, g in grads.items()}


def test_graph_replays_match_eager():
    scene, cams = _uneven()
    log("graph replay: 4 uneven views")
    ds = R.DeviceScene.from_scene(scene)
    npix = sum(c.width * c.height for c in cams)
    dl = torch.from_numpy(np.random.default_rng(2).standard_normal(3 * npix).astype(np.float32)).cuda()
    cfg = R.Config(16, 64)
    fr, g_ref = _eager(ds, cams, cfg, dl)
    img_ref = fr.images.cpu().numpy()
    P = int(fr.state.n_pairs)
    graph = R.Graph(ds, cams, R.Config(16, 64, 0, P + 1000), with_backward=True, dl_images=dl)
    for rep in range(3):
        graph.launch()
        graph.stream.synchronize()
        assert graph.status() == P
        np.testing.assert_array_equal(graph.images.cpu().numpy(), img_ref)
        for p, g in graph.grads.items():
            if g is not None:
                grad_close(f"replay {rep} {p}", g.cpu().numpy().astype(np.float64), g_ref[p].astype(np.float64),
                           rel=1e-5)
        # eager work between replays on the default stream
        _eager(ds, cams, cfg, dl)
    graph.close()


def test_graph_capture_is_the_same_call(monkeypatch):
    """megs_graph_capture (the capture step's name for megs_graph_create) builds the same graph: its
    replays give the eager forward's images bit for bit."""
    scene, cams = _uneven()
    ds = R.DeviceScene.from_scene(scene)
    fr = R.forward(ds, cams, R.Config(16, 64))
    torch.cuda.synchronize()
    lib = L.load()
    monkeypatch.setattr(lib, "megs_graph_create", lib.megs_graph_capture)
    graph = R.Graph(ds, cams, R.Config(16, 64, 0, int(fr.state.n_pairs) + 1000), with_backward=False)
    for _ in range(2):
        graph.launch()
        graph.stream.synchronize()
        np.testing.assert_array_equal(graph.images.cpu().numpy(), fr.images.cpu().numpy())
    graph.close()


def test_graph_forward_only_and_capacity_overflow():
    scene, cams = _uneven()
    ds = R.DeviceScene.from_scene(scene)
    fr = R.forward(ds, cams, R.Config(16, 64))
    torch.cuda.synchronize()
    P = int(fr.state.n_pairs)
    log(f"overflow: {P} pairs into capacity {P // 2}")
    small = R.Graph(ds, cams, R.Config(16, 64, 0, P // 2), with_backward=False)
    small.launch()
    with pytest.raises(L.MegsError) as e:
        small.status()
    assert e.value.status == L.MEGS_ERR_CAPACITY
    small.close()
    ok = R.Graph(ds, cams, R.Config(16, 64, 0, P), with_backward=False)
    ok.launch()
    assert ok.status() == P
    np.testing.assert_array_equal(ok.images.cpu().numpy(), fr.images.cpu().numpy())
    ok.close()


def test_persistent_queue_matches_one_group_per_tile():
    scene, cams = _uneven()
    ds = R.DeviceScene.from_scene(scene)
    npix = sum(c.width * c.height for c in cams)
    dl = torch.from_numpy(np.random.default_rng(3).standard_normal(3 * npix).astype(np.float32)).cuda()
    for tile, waves, sub in ((8, 1, 0), (16, 1, 0), (16, 4, 0), (32, 2, 0), (16, 1, 8), (32, 1, 8)):
        log(f"persistent tile {tile} waves {waves} subtile {sub}")
        fa, ga = _eager(ds, cams, R.Config(tile, 64, waves=waves, subtile=sub), dl)
        fb, gb = _eager(ds, cams, R.Config(tile, 64, L.MEGS_FLAG_PERSISTENT, waves=waves, subtile=sub), dl)
        np.testing.assert_array_equal(fa.images.cpu().numpy(), fb.images.cpu().numpy())
        for p in ga:
            if ga[p] is not None:
                # the two runs differ only in the order of the float atomics
                grad_close(f"persistent {p}", gb[p].astype(np.float64), ga[p].astype(np.float64))


def test_autotuner_picks_a_valid_config_with_the_same_images(tmp_path):
    scene, cams = _uneven()
    ds = R.DeviceScene.from_scene(scene)
    stats = {}
    cache = str(tmp_path / "autotune.json")
    best, table = R.autotune(ds, cams, R.Config(16, 64), reps=1, cache=cache, stats=stats)
    log(f"autotune best tile {best.tile} batch {best.batch}, sweep memory {stats['sweep_bytes']} B\n{table}")
    assert (best.tile, best.waves, best.subtile) in L.AUTOTUNE_COMBOS and best.batch in L.AUTOTUNE_BATCHES
    assert table.shape == (len(L.AUTOTUNE_COMBOS), len(L.AUTOTUNE_BATCHES))
    assert np.all(np.isfinite(table)) and np.all(table > 0)
    # the sub-tile candidates stage no batches: one timing for all four batch sizes
    for i, combo in enumerate(L.AUTOTUNE_COMBOS):
        if combo[2]:
            assert np.all(table[i] == table[i, 0])
    # the sweep holds one block of each kind at its largest size over the candidates (as megs_state_bytes
    # sizes them from each candidate's pair count), not 36 x 2 forward+backward's memory
    most = np.zeros(3, np.int64)
    for tile, waves, sub in L.AUTOTUNE_COMBOS:
        c = R.Config(tile, 64, waves=waves, subtile=sub)
        P = int(R.forward(ds, cams, c).state.n_pairs)
        m = L.MegsMemory()
        L.check(L.load().megs_state_bytes(ctypes.byref(ds.struct()), R.cameras_struct(cams), len(cams),
                                          ctypes.byref(c.struct()), P, ctypes.byref(m)))
        most = np.maximum(most, [m.frame, m.pairs, m.backward])
    assert stats["sweep_bytes"] == int(most.sum()), (stats["sweep_bytes"], most)
    # a second call finds the result in the cache (keyed by architecture and work) and times nothing
    cached, t2 = R.autotune(ds, cams, R.Config(16, 64), reps=1, cache=cache)
    assert t2 is None and (cached.tile, cached.batch, cached.waves, cached.subtile) == \
        (best.tile, best.batch, best.waves, best.subtile)
    a = R.forward(ds, cams, R.Config(16, 64)).images.cpu().numpy()
    b = R.forward(ds, cams, best).images.cpu().numpy()
    d = np.abs(a - b)
    assert (d > IMG_TOL).mean() < 1e-3 and d.max() < 1e-2


def _sampled_tiles(ranges, frac, seed):
    rng = np.random.default_rng(seed)
    pick = rng.random(ranges.shape[0]) < frac
    rs = ranges.copy()
    rs[~pick] = 0
    return pick, rs


RECORD_FIELDS = (("mean", 2, torch.float64), ("conic_o", 4, torch.float32), ("rgbd", 4, torch.float32),
                 ("radius", 1, torch.int32), ("cutoff", 1, torch.float32), ("chol", 4, torch.float64))


def _check_sampled_records(buf, scene, cams, tile, count, seed):
    """The records of a seeded sample of Gaussians, in every view, against the oracle's projection of
    the same Gaussians (read from their stored values)."""
    n, nv = scene.n, len(cams)
    idx = np.sort(np.random.default_rng(seed).choice(n, size=min(count, n), replace=False))
    sub = scene.subset(idx).widened()
    for vi, cam in enumerate(cams):
        rows = vi * n + idx
        g = {}
        for name, width, dt in RECORD_FIELDS:
            t = buf(name, width * n * nv, dt).view(n * nv, width) if width > 1 else buf(name, n * nv, dt)
            g[name] = t[torch.from_numpy(rows).to(t.device)].cpu().numpy()
        check_records(g, O.project(sub, scene.k, cam, tile))
    log(f"records of {len(idx)} sampled Gaussians in {nv} views against the oracle's projection")


def _full_size_sampled(scene, cams, cfg, frac, seed, graph=False, record_sample=20_000):
    """A full-size workload in a given launch configuration, eager or as one captured hipGraph
    (forward and backward of all views in one replay): the records of a seeded sample of Gaussians
    against the oracle's projection, the whole key table bit-exact against the oracle's (built from the
    GPU's own records); blend, blend backward and projection backward on a seeded sample of tiles (the
    loss weights vanish outside them, so the GPU's gradients come from the same pixels)."""
    tile = cfg.tile
    nv = len(cams)
    ds = R.DeviceScene.from_scene(scene)
    npix = sum(c.width * c.height for c in cams)
    # the per-field record planes are read back below: requesting them only adds their writes
    rcfg = dataclasses.replace(cfg, flags=cfg.flags | L.MEGS_FLAG_RECORD_PLANES)
    fr = R.forward(ds, cams, rcfg)
    torch.cuda.synchronize()
    P = int(fr.state.n_pairs)
    if graph:
        G = R.Graph(ds, cams, dataclasses.replace(rcfg, pair_capacity=P + P // 20 + 1024), with_backward=True)
        G.launch()
        assert G.status() == P
        np.testing.assert_array_equal(G.images.cpu().numpy(), fr.images.cpu().numpy())  # replay == eager
        state, alloc, images_flat = G.state, G.alloc, G.images
        log(f"graph: forward+backward of {nv} views in one replay, {P} pairs")
    else:
        state, alloc, images_flat = fr.state, fr.alloc, fr.images
    buf = lambda field, count, dtype: alloc.view(getattr(state, field), count, dtype)
    _check_sampled_records(buf, scene, cams, tile, record_sample, seed + 50)
    g = {"n_pairs": P}
    nr = scene.n * nv
    g["mean"] = buf("mean", 2 * nr, torch.float64).view(nr, 2).cpu().numpy()
    g["conic_o"] = buf("conic_o", 4 * nr, torch.float32).view(nr, 4).cpu().numpy()
    g["rgbd"] = buf("rgbd", 4 * nr, torch.float32).view(nr, 4).cpu().numpy()
    g["radius"] = buf("radius", nr, torch.int32).cpu().numpy()
    g["cutoff"] = buf("cutoff", nr, torch.float32).cpu().numpy()
    g["chol"] = buf("chol", 4 * nr, torch.float64).view(nr, 4).cpu().numpy()
    vals = buf("vals", P, torch.int32).cpu().numpy().view(np.uint32)
    tkeys = buf("tile_keys", P, torch.int32).cpu().numpy().view(np.uint32)
    T = int(state.n_tiles)
    ranges = buf("ranges", 2 * T, torch.int32).view(T, 2).cpu().numpy().view(np.uint32)
    rec = gpu_records(g)
    log(f"key table: {P} pairs over {nv} views")
    cnt = check_key_table(vals, ranges, rec, g["rgbd"][:, 3], cams, tile, scene.n, tile_keys=tkeys,
                          sub=cfg.subtile)
    log(f"key table against the oracle: {cnt}")
    off = O.tile_layout(cams, tile)
    pick, rs = _sampled_tiles(ranges, frac, seed)
    log(f"blend on {pick.sum()} sampled tiles")
    images = R.split_images(images_flat, cams)
    weights, checked = [], 0
    for vi, cam in enumerate(cams):
        ob = O.blend(cam, tile, rec, vals, rs[off[vi]:off[vi + 1]])
        img = images[vi].cpu().numpy().astype(np.float64)
        tx = (cam.width + tile - 1) // tile
        ys, xs = np.mgrid[0:cam.height, 0:cam.width]
        in_pick = pick[off[vi]:off[vi + 1]][(ys // tile) * tx + xs // tile]
        ok = in_pick & (ob["flag"] == 0)
        checked += int(ok.sum())
        if ok.any():
            assert np.abs(img - ob["image"])[:, ok].max() <= IMG_TOL, vi
        weights.append(S.loss_weights([cam], 21 + vi)[0] * ok[None].astype(np.float32))
    assert checked > 0.3 * frac * npix, (checked, npix)
    log(f"blend: {checked} pixels of the sampled tiles against the oracle")
    dl = torch.from_numpy(np.concatenate([w.reshape(-1) for w in weights])).cuda()
    assert dl.numel() == 3 * npix
    if graph:
        G.dl.copy_(dl)  # the graph reads dL/dimage in place at every replay
        G.launch()
        G.stream.synchronize()
        grads = G.grads
        g2 = grad2d_from_moments(backward_sums(G.alloc, G.state, 2, nr), g["chol"], rec["o"])
    else:
        nb = len(fr.alloc.blocks)
        grads = R.backward(ds, fr, dl)
        torch.cuda.synchronize()
        g2 = grad2d_from_moments(backward_sums(fr.alloc, fr.state, nb, nr), g["chol"], rec["o"])
    ref = np.zeros_like(g2)
    ref_abs = np.zeros_like(g2)
    for vi, cam in enumerate(cams):
        O.blend_backward(cam, tile, rec, vals, rs[off[vi]:off[vi + 1]], weights[vi], grad2d=ref, grad2d_abs=ref_abs)
    for c, name in enumerate(("u", "v", "a", "b", "c", "o", "r", "g", "b_col")):
        grad_close(f"grad2d[{name}]", g2[:, c], ref[:, c], abs_sum=ref_abs[:, c])
    pl = scene.widened()
    gr = O.zero_grads(pl)
    for vi, cam in enumerate(cams):
        O.project_backward(pl, scene.k, cam, tile, g2[vi * scene.n:(vi + 1) * scene.n], gr)
    for p in O.PLANES:
        if gr[p] is not None:
            grad_close(f"raw {p}", grads[p].cpu().numpy().astype(np.float64), gr[p])
    if graph:
        G.close()


def test_full_size_masked_1m_1080p_sampled():
    """The 1M-Gaussian 1080p masked workload (FP32, one view), per-tile blending at 16x16."""
    scene, cams = S.make_workload("masked_1m_1080p")
    log("full-size masked 1M 1080p, 16x16 tiles")
    _full_size_sampled(scene, cams, R.Config(16, 64), 0.02, 5)


def test_full_size_headline_in_bench_configuration():
    """The benchmark's headline: the masked 1M scene stored in FP16 (BF16 amplitudes), 8 views at
    1920x1080 on a ring, in the benchmark's launch configuration (32x32 tiles, 8x8 sub-tile
    blending)."""
    scene, _ = S.make_workload("masked_1m_1080p")
    scene16 = scene.stored("f16", "f16", "bf16")
    cams = S.ring_cameras(8, seed=5)
    log("full-size headline: FP16, 8 x 1080p, 32x32 tiles, 8x8 sub-tiles")
    _full_size_sampled(scene16, cams, R.Config(32, 64, subtile=8), 0.01, 6)


def test_full_size_clustered_200k_720p():
    """The 200k-Gaussian 720p workload at full size, in the benchmark's launch configuration."""
    scene, cams = S.make_workload("clustered_200k_720p")
    log("full-size clustered 200k 720p, 32x32 tiles, 8x8 sub-tiles")
    _full_size_sampled(scene, cams, R.Config(32, 64, subtile=8), 0.05, 7)


def test_full_size_fp16_3m_8x1080p_graph():
    """The 3M FP16/BF16 workload at full size: 8 views at 1920x1080 in one captured hipGraph, in the
    benchmark's launch configuration (sampled records, the whole key table, sampled blend and
    gradients)."""
    scene, cams = S.make_workload("fp16_3m_8x1080p")
    log("full-size fp16 3M x 8 x 1080p graph, 32x32 tiles, 8x8 sub-tiles")
    _full_size_sampled(scene, cams, R.Config(32, 64, subtile=8), 0.004, 9, graph=True)


def test_fp16_3m_subsample_all_views():
    """The 3M FP16/BF16 workload: a seeded 20k subsample, all 8 views at 1920x1080, end to end
    against the FP64 oracle reading the exact stored values."""
    scene, cams = S.make_workload("fp16_3m_8x1080p")
    idx = np.sort(np.random.default_rng(105).choice(scene.n, 20_000, replace=False))
    sub = scene.subset(idx)
    log("fp16 subsample: 20k Gaussians x 8 views")
    fwd = O.render(sub.widened(), sub.k, cams, 16)
    w = [wi * (1 - vw["flag"])[None].astype(np.float32) for wi, vw in zip(S.loss_weights(cams, 4), fwd["views"])]
    g = gpu_run(sub, cams, R.Config(16, 64), weights=w)
    worst = 0.0
    for vi in range(len(cams)):
        ok = fwd["views"][vi]["flag"] == 0
        d = np.abs(g["images"][vi] - fwd["images"][vi])[:, ok]
        worst = max(worst, float(d.max()))
    log(f"worst image error {worst:.2e}")
    assert worst <= IMG_TOL
    gr, _ = O.render_backward(sub.widened(), sub.k, cams, 16, w, fwd=fwd)
    for p in O.PLANES:
        if gr[p] is not None:
            l2 = grad_close(p, g["grads"][p], gr[p])
            log(f"  {p}: relative L2 {l2:.2e}")


def test_packed_depth_order_with_escaped_counts_full_size():
    """The depth pre-sort carries each record's tile count above its id (9 bits at 8 M records), and
    counts that do not fit take the escape value and are read back from the count array. At 8x8 tiles
    the 8-view 1M workload has records past that cap; its key table must equal the one-stage 64-bit
    sort's (which has no packing), bit for bit."""
    scene, _ = S.make_workload("masked_1m_1080p")
    ds = R.DeviceScene.from_scene(scene.stored("f16", "f16", "bf16"))
    cams = S.ring_cameras(8, seed=5)
    nr = scene.n * len(cams)
    idb = max(1, int(np.ceil(np.log2(nr))))
    cap = (1 << (32 - idb)) - 1
    log(f"packed depth order: {nr} records, {idb} id bits, count cap {cap}")
    two = R.forward(ds, cams, R.Config(8, 64, L.MEGS_FLAG_RECORD_PLANES))
    torch.cuda.synchronize()
    nt = two.buffer("ntiles", nr, torch.int32).cpu().numpy()
    assert int(nt.max()) >= cap, (int(nt.max()), cap)   # the escape path is taken
    P = int(two.state.n_pairs)
    T = int(two.state.n_tiles)
    v2 = two.buffer("vals", P, torch.int32).cpu().numpy()
    t2 = two.buffer("tile_keys", P, torch.int32).cpu().numpy()
    r2 = two.buffer("ranges", 2 * T, torch.int32).cpu().numpy()
    del two
    torch.cuda.empty_cache()
    one = R.forward(ds, cams, R.Config(8, 64, flags=L.MEGS_FLAG_ONE_STAGE_SORT))
    torch.cuda.synchronize()
    assert int(one.state.n_pairs) == P
    np.testing.assert_array_equal(one.buffer("vals", P, torch.int32).cpu().numpy(), v2)
    k1 = one.buffer("keys64", P, torch.int64).cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal((k1 >> np.uint64(32)).astype(np.uint32), t2.view(np.uint32))
    np.testing.assert_array_equal(one.buffer("ranges", 2 * T, torch.int32).cpu().numpy(), r2)


def test_batched_500k_16views_graph_autotuned():
    """The batched workload at its real shape: 500k clustered Gaussians, 16 views of uneven resolution
    (360p to 1080p) on a ring, forward and backward of all views in one hipGraph replay, at the launch
    configuration the autotuner picks; checked as the other full-size workloads (sampled records, the
    whole key table, blend and gradients on 2% of the tiles)."""
    scene, cams = S.make_workload("batched_500k_16views")
    ds = R.DeviceScene.from_scene(scene)
    best, table = R.autotune(ds, cams, R.Config(16, 64), reps=1)
    del ds
    torch.cuda.empty_cache()
    log(f"autotuned for 500k x 16 views: tile {best.tile} waves {best.waves} subtile {best.subtile} "
        f"batch {best.batch} ({float(np.nanmin(table)):.3f} ms)")
    _full_size_sampled(scene, cams, best, 0.02, 8, graph=True)

#!/usr/bin/env python3
"""Forward+backward throughput (Mpixel/s) and peak VRAM of the SG-splatting renderer on one MI355X.

Workload (synthetic, seeded): 1M clustered Gaussians with 4 SG lobes and soft primitive/lobe
masks. Two forms are measured:
  * headline `value`: parameters stored in FP16 (amplitudes in BF16), 8 views at 1920x1080 on a
    ring of radius 6, forward+backward of all views captured once in a hipGraph and replayed;
  * `plain_fp32`: the same scene in FP32, one 1920x1080 view, eager launches.
A step is one whole forward+backward of the workload's views. Inputs are resident in HBM before
the timed region. Launch configuration: the library's autotuner run on the headline workload itself
(tile size, waves per tile, sub-tile blending and batch depth; reported under config.autotune), or with
--no-autotune the given one (default 32x32 tiles for the key table, blending per 8x8 sub-tile); the
plain form uses the same launch. Each stage's kernels are also timed live with HIP events (eager calls of the same
workload); the slowest stage gives the roofline line, and every stage is set against its own bound
(`stage_roofline`: algorithmic HBM bytes at 8 TB/s, or blend FLOPs at the FP32 peak), the whole
path against the sum of those bounds (`path_roofline`). Per-step p10/p50/p90 times of the graph
come from a second run of single-step event pairs; a plain device-to-device copy gives the
achievable HBM rate (`hbm_copy`), which each HBM stage is also set against. The FP64 CPU oracle is
timed on the headline workload's views (all 8 by default), and beside it on the plain FP32 view and
on the 2,000-Gaussian 128x128 case. Also reported: the post-processing of a post-ADMM scene and an
SG-versus-SH colour comparison on the same renderer (skip with --no-post).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-post] [--no-workloads] [--no-autotune]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0        # MI355X HBM3E
PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector (packed); the unpacked FMA ceiling is half of it

# Algorithmic FP32 operations per fragment (FMA = 2, add/mul/compare/exp = 1):
#   alpha test of an evaluated fragment (offsets, quadratic form, exp, opacity, clamp, threshold): 15
#   forward blend of an included fragment (transmittance, weight, colour accumulate): 10
#   backward of an included fragment: transmittance recovery (1 - alpha, divide) 2, weight 1,
#   colour gradient 3, alpha gradient ((c - S) . dL/dC as c . dL/dC minus the carried P = S . dL/dC,
#   times T) 7, recursion of P (1 FMA) 2, opacity gradient e = G dL/dalpha 1, the five moments of e
#   (e dx, e dy, e dx^2, e dx dy, e dy^2) 5, summation of the 9 sums over pixels 9: 30 (the
#   exponent gradient is o_eff e; o_eff and the conic are applied once per record, not per fragment)
FLOP_TEST, FLOP_FWD_BLEND, FLOP_BWD_BLEND = 15, 10, 30

# HBM bytes per launch of a kernel on the headline workload, from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) scaled by what the same counters read for a plain
# copy of known size (--calibrate-copy). Each entry holds the SHA-256 of the kernel's source file
# when the counters were taken; a changed source reports traffic as null.
TRAFFIC = {
    # 1M masked Gaussians, FP16, 8 x 1920x1080, 32x32 tiles, 8x8 sub-tile blending: FETCH_SIZE
    # 2,173,650 KiB x 1.9998 (a 512 MiB copy read 262,167 KiB) + WRITE_SIZE 1,187,047 KiB x 1.0000
    "blend_bwd": {"bytes": 5666777281,
                  "source_sha256": "7c9dbb326179f52600e406b28a064c01c7630fbd32e397db7d3ae56f4519ed07"},
}
# VALU instructions per launch of the blend kernels on the same workload, from a rocprofv3 --pmc
# SQ_INSTS_VALU run (per dispatch, averaged), with the SHA-256 of the source they were taken on (a
# changed source reports them as null). At one wave64 VALU instruction per 4 cycles on each of the
# 1024 SIMDs at 2.4 GHz they give the issue time; set against the measured time it is the kernel's
# VALU utilisation.
VALU = {
    "blend_fwd": {"instructions": 512547725,
                  "source_sha256": "7c9dbb326179f52600e406b28a064c01c7630fbd32e397db7d3ae56f4519ed07"},
    "blend_bwd": {"instructions": 1196378670,
                  "source_sha256": "7c9dbb326179f52600e406b28a064c01c7630fbd32e397db7d3ae56f4519ed07"},
}
SIMDS, CLOCK_HZ, VALU_CYCLES = 1024, 2.4e9, 4
STAGE_SOURCE = {"project": "project.hip", "project_bwd": "project.hip", "blend_fwd": "blend.hip",
                "blend_bwd": "blend.hip", "depth_sort": "sort.hip", "pair_sort": "sort.hip", "scan": "sort.hip",
                "emit": "sort.hip", "ranges": "sort.hip"}


def _measured(table, stage, key):
    """table[stage][key] if it was measured on the stage's current source, else None."""
    import hashlib
    t = table.get(stage)
    if not t:
        return None
    src = os.path.join(ROOT, "paper_2509_07021_amd", "csrc", STAGE_SOURCE[stage])
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != t["source_sha256"]:
            return None
    return t[key]


def traffic_of(stage):
    return _measured(TRAFFIC, stage, "bytes")


def valu_of(stage, avg_ms):
    """VALU instructions per launch, their issue time and its share of the measured time, or None."""
    n = _measured(VALU, stage, "instructions")
    if n is None:
        return None
    issue_ms = n * VALU_CYCLES / (SIMDS * CLOCK_HZ) * 1e3
    return {"instructions": n, "issue_ms": round(issue_ms, 4), "issue_frac": round(issue_ms / avg_ms, 4)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1_000_000, help="Gaussians (default: the 1M workload)")
    ap.add_argument("--views", type=int, default=8)
    ap.add_argument("--tile", type=int, default=32)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--waves", type=int, default=0, help="wave64s per tile workgroup (0: library default)")
    ap.add_argument("--subtile", type=int, default=8,
                    help="8: blend per 8x8 sub-tile (16x16 / 32x32 tiles); 0: per tile")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use --tile/--batch/--waves/--subtile instead of the autotuner's choice for the headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-views", type=int, default=8, help="views of the workload the oracle renders")
    ap.add_argument("--no-post", action="store_true",
                    help="skip the post-processing and colour-model measurements")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the 200k 720p, 500k x 16-view and 3M x 8-view workload lines")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of MIB MiB (reference kernel for HBM counters)")
    return ap.parse_args()


def timed(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def step_percentiles(fn, steps, stream):
    """Per-step times (ms) of `steps` further launches, each bracketed by its own events."""
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for e0, e1 in evs:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    t = sorted(e0.elapsed_time(e1) for e0, e1 in evs)
    pick = lambda q: round(t[min(len(t) - 1, int(round(q * (len(t) - 1))))], 4)
    return {"p10": pick(0.1), "p50": pick(0.5), "p90": pick(0.9), "steps": steps}


def fragment_counts(R, ds, cams, cfg):
    """(blended, evaluated, replayed) fragments of one forward, counted by the stats instance."""
    import torch
    from paper_2509_07021_amd import _lib as L
    c = R.Config(cfg.tile, cfg.batch, cfg.flags | L.MEGS_FLAG_STATS, 0, cfg.waves, cfg.subtile)
    fr = R.forward(ds, cams, c)
    torch.cuda.synchronize()
    st = fr.buffer("device_status", 8, torch.int32).cpu().numpy()
    blended = int(st[4:6].view("uint64")[0])
    evaluated = int(st[6:8].view("uint64")[0])
    replayed = int(fr.buffer("last", fr.state.n_pixels, torch.int32).to(torch.int64).sum().item())
    return blended, evaluated, replayed, int(fr.state.n_pairs)


def stage_bytes(stage, n, nv, pairs, npix, ntiles, geom_bytes, k, tile_bits=14):
    """Algorithmic HBM bytes of one launch of an HBM-bound stage (two-stage sort, default flags)."""
    nr = n * nv
    rec = 48 + 4 + 4 + 4                    # packed record, tile count, depth key, sort value
    if stage == "project":
        return n * geom_bytes + nr * rec
    if stage == "depth_sort":
        return 4 * nr * (4 + 8 + 8)         # 4 passes: key read (count), key+value read, write
    if stage == "scan":
        return nr * (4 + 4 + 4 + 4)         # sorted values read twice, rewritten as ids, offsets written
    if stage == "emit":
        # order and offset per record, the record's mean, factors and opacity; key+value per pair
        return nr * (4 + 4 + 36) + pairs * 8
    if stage == "pair_sort":
        passes = (tile_bits + 7) // 8
        return passes * pairs * (4 + 8 + 8)
    if stage == "ranges":
        return pairs * 4 + ntiles * 8
    if stage == "project_bwd":
        # parameters (both passes read their planes once), the records' 9 sums and conic factors, the
        # gradient planes written
        return n * geom_bytes + nr * (9 * 4 + 16) + n * (14 + 8 * k) * 4
    return 0


def compact_bytes(scene, out_n, out_lobes):
    """Algorithmic HBM bytes of the post-processing compaction: the mark pass reads the opacity,
    mask and sharpness planes and writes a flag and a count per Gaussian; the two scans read and
    write 4 B per Gaussian each; the write pass reads every input plane once and writes the
    compacted planes, offsets and index maps."""
    eg = 4 if scene.dt_geom == "f32" else 2
    ec = 4 if scene.dt_color == "f32" else 2
    ea = 4 if scene.dt_amp == "f32" else 2
    n, k = scene.n, scene.k
    masks = scene.pmask_logit is not None
    mark = n * (eg * (1 + masks) + ec * k) + 8 * n
    scans = 2 * 2 * 4 * n
    read = n * (eg * (11 + masks) + ec * 3 + k * (ec * (4 + masks) + ea * 3)) + 12 * n
    write = out_n * (eg * 11 + ec * 3 + 8) + out_lobes * (ec * 4 + ea * 3 + 4) + 4
    return mark + scans + read + write


def post_processing(args, cfg):
    """Post-processing (Sec. 3.3) of the post-ADMM workload: compaction time, static parameter
    memory before and after, and forward+backward Mpixel/s of the dense and compacted scenes."""
    import torch
    from paper_2509_07021_amd import prune as P
    from paper_2509_07021_amd import render as R
    from paper_2509_07021_amd import scenes as S
    scene, cams = S.make_workload("post_admm_1600k_1080p")
    ds = R.DeviceScene.from_scene(scene)
    torch.cuda.synchronize()
    for _ in range(3):
        P.compact(ds, 0.01, 1.0)
    torch.cuda.synchronize()
    # the median call: a call that has to grow torch's cached device memory first (hipMalloc) takes
    # milliseconds more, which is the allocator's cost, not the compaction's
    times = []
    for _ in range(9):
        t0 = time.perf_counter()
        cds, kept, lsrc = P.compact(ds, 0.01, 1.0)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    ms_compact = sorted(times)[len(times) // 2]
    by = compact_bytes(scene, cds.n, cds.n_lobes)
    npix = sum(c.width * c.height for c in cams)
    dl = torch.randn(3 * npix, device="cuda")
    stream = torch.cuda.current_stream()
    rates = {}
    for name, d in (("dense", ds), ("compacted", cds)):
        ms = timed(lambda: R.backward(d, R.forward(d, cams, cfg), dl), args.steps, args.warmup, stream)
        rates[name] = {"ms_per_step": round(ms, 4), "Mpixel/s": round(npix / ms / 1e3, 2),
                       "static_params_mb": round(d.static_bytes() / 1e6, 1)}
    lobes_per = cds.n_lobes / max(cds.n, 1)
    log(f"post-processing: {scene.n} -> {cds.n} Gaussians, {cds.n_lobes} lobes ({lobes_per:.3f}/Gaussian), "
        f"compaction {ms_compact:.3f} ms, dense {rates['dense']['Mpixel/s']} vs compacted "
        f"{rates['compacted']['Mpixel/s']} Mpixel/s")
    return {"workload": (f"{scene.n} clustered Gaussians, {scene.k} SG lobes, soft masks, FP32, post-ADMM state "
                         f"(40% near-zero opacity, 68% of lobes with sharpness < 1); thresholds opacity 0.01, "
                         f"sharpness 1; 1 view 1920x1080"),
            "gaussians_in": scene.n, "gaussians_out": cds.n, "lobes_out": cds.n_lobes,
            "lobes_per_gaussian": round(lobes_per, 4), "colour_floats_per_gaussian": round(3 + 7 * lobes_per, 3),
            "compact_ms": round(ms_compact, 4),
            "compact_note": "median wall time of 9 calls, each including its one host synchronisation",
            "compact_algorithmic_bytes": by, "compact_GBps": round(by / (ms_compact * 1e-3) / 1e9, 1),
            "render": rates}


def colour_models(args, cfg, scene, cams):
    """Same renderer, same geometry, two colour models: SG with 3 lobes (24 colour floats per
    Gaussian, the paper's model before lobe pruning) and degree-3 spherical harmonics (48 floats,
    3DGS's model). FP32, one view, eager forward+backward; static parameter bytes and Mpixel/s."""
    import dataclasses
    import torch
    from paper_2509_07021_amd import render as R
    from paper_2509_07021_amd import scenes as S
    base = dataclasses.replace(scene, pmask_logit=None, lmask_logit=None)
    sg3 = dataclasses.replace(base, k=3, axis=base.axis[:3].copy(), sharp=base.sharp[:3].copy(),
                              amp=base.amp[:3].copy())
    sh3 = S.sh_scene(base, 3, 3)
    npix = sum(c.width * c.height for c in cams)
    dl = torch.randn(3 * npix, device="cuda")
    stream = torch.cuda.current_stream()
    out = {}
    for name, sc in (("sg_3_lobes", sg3), ("sh_degree_3", sh3)):
        ds = R.DeviceScene.from_scene(sc)
        ms = timed(lambda: R.backward(ds, R.forward(ds, cams, cfg), dl), args.steps, args.warmup, stream)
        with R.Profile() as prof:
            R.backward(ds, R.forward(ds, cams, cfg), dl)
        out[name] = {"ms_per_step": round(ms, 4), "Mpixel/s": round(npix / ms / 1e3, 2),
                     "static_params_mb": round(ds.static_bytes() / 1e6, 1),
                     "project_ms": round(prof.ms["project"], 4), "project_bwd_ms": round(prof.ms["project_bwd"], 4)}
        del ds
        torch.cuda.empty_cache()
    log("colour models: " + ", ".join(f"{k} {v['Mpixel/s']} Mpixel/s {v['static_params_mb']} MB" for k, v in out.items()))
    out["workload"] = f"{scene.n} clustered Gaussians (no masks), FP32, 1 view 1920x1080, eager forward+backward"
    return out


def oracle_seconds(scene, cams, tile, seed=11):
    """(forward s, backward s, pixels) of one full FP64 oracle forward and backward (projection,
    key table, blend, blend backward, projection backward) of `cams`, reading the exact stored
    values of `scene`."""
    from oracle import oracle as O
    from paper_2509_07021_amd import scenes as S
    pl = scene.widened()
    w = S.loss_weights(cams, seed)
    t0 = time.perf_counter()
    fwd = O.render(pl, scene.k, cams, tile)
    t1 = time.perf_counter()
    O.render_backward(pl, scene.k, cams, tile, w, fwd=fwd)
    t2 = time.perf_counter()
    return t1 - t0, t2 - t1, sum(c.width * c.height for c in cams)


def cpu_baseline(scene, cams, tile, n_sample_views, others=()):
    """The FP64 oracle on the host, on the benchmark's own workload: full forward and backward of
    the first n_sample_views of its views at full resolution, reading the exact stored (FP16/BF16)
    values. Mpixel/s of that sample is the oracle's rate for the whole step. `others` are
    (name, scene, cameras, tile) workloads timed the same way and reported beside it."""
    from oracle import oracle as O
    sample = list(cams[:n_sample_views])
    tf, tb, npix = oracle_seconds(scene, sample, tile)
    also = {}
    for name, sc, cm, tl in others:
        f, b, n = oracle_seconds(sc, list(cm), tl)
        also[name] = {"value": round(n / (f + b) / 1e6, 4), "unit": "Mpixel/s",
                      "seconds": {"forward": round(f, 3), "backward": round(b, 3)}}
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(npix / (tf + tb) / 1e6, 4), "unit": "Mpixel/s", "cores": O.threads(), "kind": "oracle",
            "cpu_model": model,
            "sample": (f"FP64 oracle on {len(sample)} of the {len(cams)} views of the benchmark workload "
                       f"({sample[0].width}x{sample[0].height}, full frames, {scene.n} Gaussians read from their "
                       f"{scene.dt_geom}/{scene.dt_color}/{scene.dt_amp} storage): forward {tf:.1f} s, "
                       f"backward {tb:.1f} s"),
            "seconds": {"forward": round(tf, 2), "backward": round(tb, 2)},
            "other_workloads": also}


def copy_rate(stream, mib=1024, reps=10):
    """Achievable HBM rate of a plain device-to-device copy of `mib` MiB (bytes read + written per
    second, GB/s), timed with HIP events: the practical ceiling the HBM-bound stages are also set
    against, beside the 8 TB/s of the specification."""
    import torch
    src = torch.ones(mib * (1 << 20) // 4, device="cuda")
    dst = torch.empty_like(src)
    ms = timed(lambda: dst.copy_(src), reps, 2, stream)
    del src, dst
    torch.cuda.empty_cache()
    return {"GBps": round(2 * mib * (1 << 20) / (ms * 1e-3) / 1e9, 1), "bytes_per_copy": 2 * mib * (1 << 20),
            "ms_per_copy": round(ms, 4)}


def stage_rooflines(R, L, ds, cams, cfg, scene, geom_bytes, pairs, hbm_copy, steps):
    """Per-stage milliseconds of eager forward+backward calls (HIP events), the dominant kernel's
    roofline line, every stage against its own bound (HBM bytes at 8 TB/s, or blend FLOPs at the FP32
    peak), and the whole path against the sum of those bounds."""
    import torch
    npix = sum(c.width * c.height for c in cams)
    dl = torch.randn(3 * npix, device="cuda")
    prof_steps = max(2, min(steps, 5))
    for _ in range(2):
        R.backward(ds, R.forward(ds, cams, cfg), dl)
    torch.cuda.synchronize()
    with R.Profile() as prof:
        for _ in range(prof_steps):
            R.backward(ds, R.forward(ds, cams, cfg), dl)
    stage_ms = {s: prof.ms[s] / max(prof.count[s], 1) for s in L.STAGES if prof.count[s]}
    blended, evaluated, replayed, _ = fragment_counts(R, ds, cams, cfg)
    dominant = max(stage_ms, key=stage_ms.get)
    nt = sum(((c.width + cfg.tile - 1) // cfg.tile) * ((c.height + cfg.tile - 1) // cfg.tile) for c in cams)
    tile_bits = max(1, (nt - 1).bit_length())
    if dominant in ("blend_fwd", "blend_bwd"):
        # the backward re-tests the fragments the forward tested (the same culled lists, walked
        # back from each pixel's last index) and differentiates the blended ones
        flops = (FLOP_TEST * evaluated + FLOP_FWD_BLEND * blended if dominant == "blend_fwd"
                 else FLOP_TEST * evaluated + FLOP_BWD_BLEND * blended)
        achieved = flops / (stage_ms[dominant] * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": dominant, "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": traffic_of(dominant),
                "units_per_launch": {"blended": blended, "evaluated": evaluated, "replayed": replayed},
                "avg_ms": round(stage_ms[dominant], 4), "valu": valu_of(dominant, stage_ms[dominant])}
    else:
        by = stage_bytes(dominant, scene.n, len(cams), pairs, npix, nt, geom_bytes, scene.k, tile_bits)
        achieved = by / (stage_ms[dominant] * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic_of(dominant),
                "avg_ms": round(stage_ms[dominant], 4)}
    stage_roof, bound_ms = {}, 0.0
    for st, ms in stage_ms.items():
        if st in ("blend_fwd", "blend_bwd"):
            fl = FLOP_TEST * evaluated + (FLOP_FWD_BLEND if st == "blend_fwd" else FLOP_BWD_BLEND) * blended
            ach = fl / (ms * 1e-3) / 1e12
            v = valu_of(st, ms)
            stage_roof[st] = {"bound": "alu", "achieved": round(ach, 2), "unit": "TFLOP/s",
                              "frac": round(ach / PEAK_FP32_TFLOPS, 4),
                              "valu_issue_frac": v["issue_frac"] if v else None}
            bound_ms += fl / (PEAK_FP32_TFLOPS * 1e12) * 1e3
        else:
            by = stage_bytes(st, scene.n, len(cams), pairs, npix, nt, geom_bytes, scene.k, tile_bits)
            ach = by / (ms * 1e-3) / 1e9
            stage_roof[st] = {"bound": "hbm", "achieved": round(ach, 1), "unit": "GB/s",
                              "frac": round(ach / PEAK_HBM_GBS, 4), "frac_of_copy": round(ach / hbm_copy["GBps"], 4),
                              "bytes": int(by)}
            bound_ms += by / (PEAK_HBM_GBS * 1e9) * 1e3
    path_roof = {"bound_ms": round(bound_ms, 4), "measured_ms": round(sum(stage_ms.values()), 4),
                 "frac": round(bound_ms / sum(stage_ms.values()), 4)}
    del dl
    return stage_ms, roof, stage_roof, path_roof


def workload_line(args, name, cfg, graph, hbm_copy, autotune=False):
    """One more workload at its full size: forward+backward Mpixel/s (eager calls, or one hipGraph replay
    of all views), peak VRAM (forward only and forward+backward), the per-view dynamic part, and the
    dominant kernel's roofline line. With autotune, the launch configuration is the autotuner's."""
    import torch
    from paper_2509_07021_amd import _lib as L
    from paper_2509_07021_amd import render as R
    from paper_2509_07021_amd import scenes as S
    t0 = time.perf_counter()
    scene, cams = S.make_workload(name)
    ds = R.DeviceScene.from_scene(scene)
    npix = sum(c.width * c.height for c in cams)
    dl = torch.randn(3 * npix, device="cuda")
    tune = None
    if autotune:
        stats = {}
        cfg, table = R.autotune(ds, cams, R.Config(16, 64), reps=1, dl_images=dl, stats=stats)
        tune = {"tile": cfg.tile, "waves": cfg.waves, "subtile": cfg.subtile, "batch": cfg.batch,
                "best_ms": round(float(table.min()), 4), "sweep_vram_mb": round(stats["sweep_bytes"] / 1e6, 1)}
        torch.cuda.empty_cache()
    stream = torch.cuda.current_stream()
    fr = R.forward(ds, cams, cfg)
    torch.cuda.synchronize()
    pairs = int(fr.state.n_pairs)
    del fr
    torch.cuda.empty_cache()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    if graph:
        gcfg = R.Config(cfg.tile, cfg.batch, cfg.flags, int(pairs * 1.02) + 4096, cfg.waves, cfg.subtile)
        gf = R.Graph(ds, cams, gcfg, with_backward=False)
        gf.launch()
        torch.cuda.synchronize()
        fwd_peak = torch.cuda.max_memory_allocated()
        gf.close()
        del gf
        torch.cuda.empty_cache()
        torch.cuda.reset_peak_memory_stats()
        g = R.Graph(ds, cams, gcfg, with_backward=True, dl_images=dl)
        g.launch()
        torch.cuda.synchronize()
        fb_peak = torch.cuda.max_memory_allocated()
        ms = timed(g.launch, args.steps, args.warmup, g.stream)
        assert g.status() == pairs
        g.close()
        del g
    else:
        fr = R.forward(ds, cams, cfg)
        torch.cuda.synchronize()
        fwd_peak = torch.cuda.max_memory_allocated()
        R.backward(ds, fr, dl)
        torch.cuda.synchronize()
        fb_peak = torch.cuda.max_memory_allocated()
        del fr

        def step():
            R.backward(ds, R.forward(ds, cams, cfg), dl)
        ms = timed(step, args.steps, args.warmup, stream)
    torch.cuda.empty_cache()
    static = ds.static_bytes()
    _, roof, _, path_roof = stage_rooflines(R, L, ds, cams, cfg, scene, static // scene.n, pairs, hbm_copy,
                                            args.steps)
    # the traffic and VALU counts are the headline workload's (measured offline on its source): not this one's
    roof["traffic"] = None
    roof["valu"] = None
    mpix = npix / ms / 1e3
    res = sorted({f"{c.width}x{c.height}" for c in cams})
    log(f"{name}: {ms:.3f} ms/step, {mpix:.1f} Mpixel/s, pairs {pairs}, fwd+bwd peak {fb_peak / 1e6:.0f} MB "
        f"({time.perf_counter() - t0:.1f}s)")
    out = {"value": round(mpix, 2), "unit": "Mpixel/s", "ms_per_step": round(ms, 4),
           "workload": (f"{scene.n} clustered Gaussians, {scene.k} SG lobes, "
                        f"{scene.dt_geom}/{scene.dt_color}/{scene.dt_amp} storage, {len(cams)} view(s) "
                        f"{'/'.join(res)}, forward+backward {'in one hipGraph' if graph else 'eager'}"),
           "gaussians": scene.n, "views": len(cams), "pixels": npix, "pairs": pairs,
           "launch": {"tile": cfg.tile, "batch": cfg.batch, "waves": cfg.waves, "subtile": cfg.subtile},
           "peak_vram_mb": {"forward": round(fwd_peak / 1e6, 1), "forward_backward": round(fb_peak / 1e6, 1),
                            "static_params": round(static / 1e6, 1), "resident_before": round(before / 1e6, 1),
                            "dynamic_per_view": round((fb_peak - before) / len(cams) / 1e6, 1)},
           "roofline": roof, "path_roofline": path_roof}
    if tune:
        out["autotune"] = tune
    del ds, dl
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the multi-GPU design is view sharding with one gradient all-reduce, not built).",
              file=sys.stderr)
        return 2
    import numpy as np
    import torch
    from paper_2509_07021_amd import _lib as L
    from paper_2509_07021_amd import render as R
    from paper_2509_07021_amd import scenes as S

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy * (1 << 20) // 4, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calibrate_copy} MiB read + {args.calibrate_copy} MiB written")
        del src, dst
    hbm_copy = copy_rate(torch.cuda.current_stream())
    log(f"plain copy: {hbm_copy['GBps']:.0f} GB/s")
    t_start = time.perf_counter()
    scene, cams1 = S.make_workload("masked_1m_1080p", n=args.n)
    scene16 = scene.stored("f16", "f16", "bf16")
    cams8 = S.ring_cameras(args.views, seed=5)
    log(f"scenes ready in {time.perf_counter() - t_start:.1f}s: n={scene.n} k={scene.k}")
    cfg = R.Config(args.tile, args.batch, waves=args.waves, subtile=args.subtile)
    tuned = None
    if not args.no_autotune:
        # the launch configuration: the library's autotuner on the headline workload itself (every
        # tile size, waves per tile and sub-tile blending x batch depth, timed forward+backward)
        ds16 = R.DeviceScene.from_scene(scene16)
        dl8 = torch.randn(3 * sum(c.width * c.height for c in cams8), device="cuda")
        stats = {}
        t0 = time.perf_counter()
        cfg, table = R.autotune(ds16, cams8, R.Config(16, 64), reps=1, dl_images=dl8, stats=stats)
        tuned = {"tile": cfg.tile, "waves": cfg.waves, "subtile": cfg.subtile, "batch": cfg.batch,
                 "best_ms": round(float(table.min()), 4), "sweep_s": round(time.perf_counter() - t0, 2),
                 "sweep_vram_mb": round(stats["sweep_bytes"] / 1e6, 1)}
        log(f"autotune: tile {cfg.tile} waves {cfg.waves} subtile {cfg.subtile} batch {cfg.batch} "
            f"in {tuned['sweep_s']} s; ms per (tile, waves, subtile) x batch:\n{table}")
        del ds16, dl8
        torch.cuda.empty_cache()

    # ---------------------------------------------------------------- plain FP32, 1 view (same launch)
    ds = R.DeviceScene.from_scene(scene)
    npix1 = sum(c.width * c.height for c in cams1)
    dl1 = torch.randn(3 * npix1, device="cuda")
    stream = torch.cuda.current_stream()

    def step_plain():
        fr = R.forward(ds, cams1, cfg)
        R.backward(ds, fr, dl1)

    torch.cuda.synchronize()
    base_alloc = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    fr = R.forward(ds, cams1, cfg)
    torch.cuda.synchronize()
    plain_fwd_peak = torch.cuda.max_memory_allocated()
    R.backward(ds, fr, dl1)
    torch.cuda.synchronize()
    plain_fb_peak = torch.cuda.max_memory_allocated()
    plain_pairs = int(fr.state.n_pairs)
    del fr
    ms_plain = timed(step_plain, args.steps, args.warmup, stream)
    log(f"plain fp32: {ms_plain:.3f} ms/step, {npix1 / ms_plain / 1e3:.1f} Mpixel/s, pairs {plain_pairs}")

    # ---------------------------------------------------------------- FP16 batched graph, 8 views
    del ds
    torch.cuda.empty_cache()
    ds16 = R.DeviceScene.from_scene(scene16)
    static16 = ds16.static_bytes()
    npix8 = sum(c.width * c.height for c in cams8)
    dl8 = torch.randn(3 * npix8, device="cuda")
    fr = R.forward(ds16, cams8, cfg)
    torch.cuda.synchronize()
    pairs8 = int(fr.state.n_pairs)
    del fr
    torch.cuda.empty_cache()
    cap = int(pairs8 * 1.02) + 4096
    gcfg = R.Config(cfg.tile, cfg.batch, cfg.flags, cap, cfg.waves, cfg.subtile)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    gf = R.Graph(ds16, cams8, gcfg, with_backward=False)
    gf.launch()
    torch.cuda.synchronize()
    batched_fwd_peak = torch.cuda.max_memory_allocated()
    gf.close()
    del gf
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    g = R.Graph(ds16, cams8, gcfg, with_backward=True, dl_images=dl8)
    g.launch()
    torch.cuda.synchronize()
    batched_fb_peak = torch.cuda.max_memory_allocated()
    counted = g.status()
    ms_batched = timed(g.launch, args.steps, args.warmup, g.stream)
    step_ms = step_percentiles(g.launch, max(args.steps, 10), g.stream)
    counted_after = g.status()
    assert counted == counted_after == pairs8, (counted, counted_after, pairs8)
    mpix_batched = npix8 / ms_batched / 1e3
    log(f"fp16 batched graph: {ms_batched:.3f} ms/step, {mpix_batched:.1f} Mpixel/s, pairs {pairs8}")
    g.close()
    del g
    torch.cuda.empty_cache()

    # ---------------------------------------------------------------- per-stage timing, same workload
    geom_bytes = static16 // scene.n
    stage_ms, roof, stage_roof, path_roof = stage_rooflines(R, L, ds16, cams8, cfg, scene, geom_bytes, pairs8,
                                                            hbm_copy, args.steps)
    log("stage ms: " + ", ".join(f"{k} {v:.3f}" for k, v in stage_ms.items()))
    dyn_per_view = (batched_fb_peak - before) / len(cams8)

    out = {
        "metric": "fwd+bwd Mpixel/s at 1M Gaussians 1080p, peak VRAM; FP16-batched vs FP32 plain",
        "value": round(mpix_batched, 2),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_batched, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"{scene.n} clustered Gaussians, {scene.k} SG lobes, soft masks, FP16 storage "
                                f"(BF16 amplitudes), {len(cams8)} views 1920x1080, forward+backward in one hipGraph"),
                   "gaussians": scene.n, "views": len(cams8), "resolution": "1920x1080", "tile": cfg.tile,
                   "batch": cfg.batch, "waves": cfg.waves, "subtile": cfg.subtile, "storage": "f16/f16/bf16",
                   "pairs": pairs8, "autotune": tuned},
        "peak_vram_mb": {"forward": round(batched_fwd_peak / 1e6, 1), "forward_backward": round(batched_fb_peak / 1e6, 1),
                         "static_params": round(static16 / 1e6, 1), "resident_before": round(before / 1e6, 1),
                         "dynamic_per_view": round(dyn_per_view / 1e6, 1)},
        "plain_fp32": {"value": round(npix1 / ms_plain / 1e3, 2), "unit": "Mpixel/s", "ms_per_step": round(ms_plain, 4),
                       "workload": f"{scene.n} clustered Gaussians, FP32, 1 view 1920x1080, eager",
                       "pairs": plain_pairs,
                       "peak_vram_mb": {"forward": round((plain_fwd_peak) / 1e6, 1),
                                        "forward_backward": round(plain_fb_peak / 1e6, 1),
                                        "static_params": round(scene.n * (14 + 8 * scene.k + 1) * 4 / 1e6, 1),
                                        "resident_before": round(base_alloc / 1e6, 1)}},
        "step_ms_percentiles": step_ms,
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "stage_roofline": stage_roof,
        "path_roofline": path_roof,
        "roofline": roof,
        "hbm_copy": hbm_copy,
    }
    del ds16
    torch.cuda.empty_cache()
    if not args.no_post:
        out["post_processing"] = post_processing(args, cfg)
        out["colour_models"] = colour_models(args, cfg, scene, cams1)
    if not args.no_workloads:
        out["workloads"] = {
            "clustered_200k_720p": workload_line(args, "clustered_200k_720p", cfg, False, hbm_copy),
            "batched_500k_16views": workload_line(args, "batched_500k_16views", cfg, True, hbm_copy, autotune=True),
            "fp16_3m_8x1080p": workload_line(args, "fp16_3m_8x1080p", cfg, True, hbm_copy),
        }
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        small, cams_small = S.make_workload("small_2k_128px")
        others = [("masked_1m_1080p FP32, 1 view (the plain form)", scene, cams1, cfg.tile),
                  ("small_2k_128px FP32, 1 view 128x128, 16x16 tiles", small, cams_small, 16)]
        out["cpu_baseline"] = cpu_baseline(scene16, cams8, cfg.tile, args.cpu_views, others)
        log(f"cpu baseline in {time.perf_counter() - t0:.1f}s")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

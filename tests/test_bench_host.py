"""Host logic of bench.py, on the CPU: the refusal of more than one GPU, the rule that a stored HBM
traffic figure is reported only for the kernel source it was measured on, the algorithmic bytes per
stage, and the structure of the oracle's CPU baseline on a small workload."""
import hashlib
import json
import os
import subprocess
import sys

import bench

STAGES_HBM = ("project", "depth_sort", "scan", "emit", "pair_sort", "ranges", "project_bwd")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no bench line


def test_traffic_is_reported_only_for_the_source_it_was_measured_on(monkeypatch):
    src = os.path.join(bench.ROOT, "paper_2509_07021_amd", "csrc", "blend.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    monkeypatch.setitem(bench.TRAFFIC, "blend_bwd", {"bytes": 123, "source_sha256": sha})
    assert bench.traffic_of("blend_bwd") == 123
    monkeypatch.setitem(bench.TRAFFIC, "blend_bwd", {"bytes": 123, "source_sha256": "0" * 64})
    assert bench.traffic_of("blend_bwd") is None
    assert "emit" not in bench.TRAFFIC and bench.traffic_of("emit") is None


def test_valu_issue_time_is_reported_only_for_the_measured_source(monkeypatch):
    src = os.path.join(bench.ROOT, "paper_2509_07021_amd", "csrc", "blend.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    n = 1024 * 2_400_000 // 4  # one millisecond of issue: 1024 SIMDs x 2.4e9 cycles x 1e-3 / 4 cycles
    monkeypatch.setitem(bench.VALU, "blend_bwd", {"instructions": n, "source_sha256": sha})
    v = bench.valu_of("blend_bwd", 2.0)
    assert v["instructions"] == n and v["issue_ms"] == 1.0 and v["issue_frac"] == 0.5
    monkeypatch.setitem(bench.VALU, "blend_bwd", {"instructions": n, "source_sha256": "0" * 64})
    assert bench.valu_of("blend_bwd", 2.0) is None


def test_stage_bytes_follow_the_per_unit_counts():
    n, nv, pairs, npix, ntiles, gb, k = 1000, 8, 40_000, 8 * 1920 * 1080, 16_320, 94, 4
    nr = n * nv
    args = (n, nv, pairs, npix, ntiles, gb, k)
    for st in STAGES_HBM:
        assert bench.stage_bytes(st, *args) > 0, st
    assert bench.stage_bytes("blend_bwd", *args) == 0  # the blends are counted in FLOPs
    # parameters read once, per view a 48-byte record, its tile count, depth key and sort value
    assert bench.stage_bytes("project", *args) == n * gb + nr * 60
    # order, offset and 36 bytes of the record per record; key and value per pair
    assert bench.stage_bytes("emit", *args) == nr * 44 + pairs * 8
    # one radix pass per 8 tile bits, each reading the keys twice and the values once, writing both
    assert bench.stage_bytes("pair_sort", *args, tile_bits=14) == 2 * pairs * 20
    assert bench.stage_bytes("pair_sort", *args, tile_bits=8) == pairs * 20
    assert bench.stage_bytes("ranges", *args) == pairs * 4 + ntiles * 8
    # the headline's pair sort moves more than its depth sort, which moves more than the scan
    big = (1_000_000, 8, 31_816_257, npix, ntiles, gb, k)
    assert bench.stage_bytes("pair_sort", *big) > bench.stage_bytes("depth_sort", *big) > bench.stage_bytes("scan", *big)


def test_cpu_baseline_reports_the_oracle_on_its_sample_and_beside_it(oracle):
    from paper_2509_07021_amd import scenes as S
    sc, cams = S.make_workload("small_2k_128px")
    out = bench.cpu_baseline(sc, list(cams), 16, 1, others=[("the same case again", sc, list(cams), 16)])
    assert out["kind"] == "oracle" and out["unit"] == "Mpixel/s"
    assert out["value"] > 0 and out["cores"] >= 1
    assert "1 of the 1 views" in out["sample"] and "f32/f32/f32" in out["sample"]
    assert set(out["other_workloads"]) == {"the same case again"}
    other = out["other_workloads"]["the same case again"]
    assert other["unit"] == "Mpixel/s" and other["value"] > 0
    assert other["seconds"]["forward"] >= 0 and other["seconds"]["backward"] >= 0
    json.dumps(out)  # it goes into the bench line as it is

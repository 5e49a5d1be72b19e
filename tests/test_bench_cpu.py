"""bench.py pieces that need no GPU: the one-GPU guard, the counter record
lookup and the VALU fraction."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_record_applies_only_to_its_sources_and_config():
    with open(bench.TRAFFIC_FILE) as f:
        rec = json.load(f)
    cfg = rec["config"]
    if rec["source_sha1"] == bench.kernel_source_sha1():
        assert bench.recorded_traffic(cfg) == rec["traffic_bytes_per_launch"]
    else:
        assert bench.recorded_traffic(cfg) is None
    # filed under the key the default bench run looks up (H, FP32, quad, occupancy)
    assert cfg == bench.counter_config("H", "f32", "quad", True)
    other = dict(cfg, dtype="bf16")
    assert bench.recorded_traffic(other) is None
    assert bench.recorded_counters(other) == {}


def test_valu_fraction():
    assert bench.valu_fraction({}, 0.2) is None
    v = bench.valu_fraction({"valu_insts_per_launch": 1_000_000}, 1.0)
    # 1e6 wave instructions x 64 lanes in 1 ms, against 256 x 64 x 2.4e9 lane-instr/s
    assert abs(v["frac"] - 64e9 / (256 * 64 * 2.4e9)) < 1e-4
    assert v["peak"] == round(256 * 64 * 2.4e9 / 1e12, 2)


def test_oracle_subset_counts_the_subset_lookups():
    from oracle import cloud as O
    from paper_1609_05344_amd import scenes
    r = bench.oracle_subset("C1", "f32", 128, 0, 64, 2)
    w = scenes.workload("C1")
    sc = scenes.make_scene(w, dtype="f32")
    vol = O.OracleVolume(base=sc.base_f64)
    pix = scenes.random_pixels(w.width, w.height, 64, seed=4096)
    _, lk = O.render(vol, w.camera(0), w.params, w.width, w.height, frame=0, pixels=pix,
                     return_lookups=True)
    assert r["pixels"] == 64 and r["lookups"] == lk and r["steps"] == 128

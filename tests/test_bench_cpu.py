"""bench.py pieces that need no GPU: the one-GPU guard, the counter record
lookup, the roofline object and the fixed timed window."""

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
    got = bench.recorded_counters(cfg).get("traffic_bytes_per_launch")
    if rec["source_sha1"] == bench.kernel_source_sha1():
        assert got == rec["traffic_bytes_per_launch"]
    else:
        assert got is None
    # filed under the key the default bench run looks up (H, FP32, quad, occupancy)
    assert cfg == bench.counter_config("H", "f32", "quad", True)
    other = dict(cfg, dtype="bf16")
    assert bench.recorded_counters(other) == {}


def test_roofline_fractions():
    alg = {"ops_per_launch": 3.0e9, "units_per_launch": {}, "ops_per_unit": {}}
    rec = {"traffic_bytes_per_launch": 800_000_000, "valu_insts_per_launch": 50_000_000}
    r = bench.roofline(rec, alg, 0.2, 1e6, 32)
    peak = 256 * 64 * 2.4e9
    # 3e9 lane operations in 0.2 ms against 256 x 64 x 2.4e9 per second
    assert r["bound"] == "alu" and abs(r["frac"] - 3e9 / 2e-4 / peak) < 1e-4
    assert abs(r["achieved"] - 3e9 / 2e-4 / 1e12) < 1e-3
    assert abs(r["hbm"]["frac"] - 8e8 / 2e-4 / 8e12) < 1e-4
    assert abs(r["valu_issued"]["frac"] - 5e7 * 64 / 2e-4 / peak) < 1e-4
    assert r["traffic"] == 800_000_000
    empty = bench.roofline({}, None, 0.2, 1e6, 32)
    assert empty["frac"] is None and empty["hbm"] is None and empty["valu_issued"] is None


def test_timed_window_does_not_depend_on_warmup_or_steps():
    # a short run (--steps 20 --warmup 5) and the defaults time the same frames
    a, b = bench.timed_frames(20), bench.timed_frames(300)
    assert sorted(set(a)) == sorted(set(b)) == list(range(bench.TIMED_FIRST,
                                                          bench.TIMED_FIRST + bench.TIMED_PERIOD))
    assert all(b.count(f) == 300 // bench.TIMED_PERIOD for f in set(b))
    assert bench.warm_frames(5) == list(range(bench.TIMED_FIRST - 5, bench.TIMED_FIRST))
    assert bench.warm_frames(200)[-1] == bench.TIMED_FIRST - 1
    big = bench.warm_frames(bench.TIMED_FIRST + 7)
    assert min(big) >= 0 and max(big) < bench.TIMED_FIRST and big[-1] == bench.TIMED_FIRST - 1


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


def test_event_sample_covers_the_window():
    """Timing events go on a sample of the timed steps: distinct, in order,
    starting at the first step, about one in EVENT_EVERY, and over a long run
    every frame of the timed window is among them."""
    for steps in (1, 5, 20, 21, 300, 1000):
        s = bench.event_steps(steps)
        assert s[0] == 0 and s == sorted(set(s)) and s[-1] < steps
        assert abs(len(s) - len(range(0, steps, bench.EVENT_EVERY))) <= 1
    frames = [bench.timed_frames(300)[k] for k in bench.event_steps(300)]
    assert set(frames) == set(bench.timed_frames(bench.TIMED_PERIOD))

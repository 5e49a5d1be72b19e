#!/usr/bin/env python3
"""Benchmark of the cloud raymarch hot path on one MI355X.

One step = one frame of the whole hot path at 1920x1080: per-pixel primary
march with a jittered start (8 steps), a 6-step light march per sample, phase
plus ambient, analytic step integration (one render launch), then the
3x3-clamped temporal resolve into the history (one resolve launch). The
camera orbits one degree per frame, as in the paper's moving-scene use.

    python bench.py [--gpus 1] [--steps 300] [--warmup 200]

Prints one JSON line. `value` is executed trilinear density lookups per
second (Gsamples/s) over the timed frames, inputs resident in HBM; the
per-frame lookup count comes from the library's own counter (not timed).
"""

from __future__ import annotations

import argparse
import ctypes
import gc
import json
import math
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X_HBM_GBPS = 8000.0
# FP32 vector issue peak without packed math: 256 CUs x 64 lanes x 2.4 GHz
MI355X_VALU_LANE_INSTR_PER_S = 256 * 64 * 2.4e9
MI355X_FP32_VECTOR_TFLOPS = 157.3
KERNEL_SOURCES = ["cloud_device.h", "cloud_types.h", "render.hip"]
# Timed frames: orbit frames TIMED_FIRST .. TIMED_FIRST + TIMED_PERIOD - 1,
# cycled, so that the work per timed frame does not depend on --warmup or on
# --steps (for a multiple of TIMED_PERIOD).
TIMED_FIRST = 400
TIMED_PERIOD = 20
# untimed frames before the timed ones, at least (warm-up plus settling)
SETTLE_FRAMES = 200
# timed steps that carry timing events (every EVENT_EVERY-th, from the first):
# an event is a packet between kernels that costs 1-2 us, so the others go
# without
EVENT_EVERY = 4
# Arithmetic type of the path for each storage type: every optical depth,
# transmittance, exponential and colour is float32; 16-bit storage adds
# 16-bit texels (and, for FP16, 16-bit x-lerp weights in dot products).
PATH_DTYPE = {"f32": "f32", "f16": "f16-storage/f32", "bf16": "bf16-storage/f32"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "render_traffic.json")


JITTER_NAMES = {0: "none (j = 1/2)", 1: "per-pixel", 2: "per 8x8 tile", 3: "per frame"}


def kernel_source_sha1() -> str:
    """Hash of the sources the render kernel is built from: a recorded counter
    measurement applies only while this hash is unchanged."""
    import hashlib
    h = hashlib.sha1()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1609_05344_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded_counters(config: dict) -> dict:
    """The committed rocprofv3 measurement of the render kernel (HBM bytes per
    launch from FETCH_SIZE / WRITE_SIZE, VALU instructions per launch from
    SQ_INSTS_VALU), or {} when the kernel sources or the config differ."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return {}
    if rec.get("source_sha1") != kernel_source_sha1() or rec.get("config") != config:
        return {}
    return rec


# ---------------------------------------------------------------------------
# Timing events
# ---------------------------------------------------------------------------

_HIP = None


class TimingEvent:
    """A HIP timing event on torch's current stream (the stream the library
    launches on), recorded without the system-scope fence
    (hipEventDisableSystemFence). A default event writes back and invalidates
    the caches when it completes, which adds about 1.7 us a record at 1080p and
    slows the kernel after it. Read only after a device-wide synchronize."""
    DISABLE_SYSTEM_FENCE = 0x20000000

    def __init__(self):
        global _HIP
        import torch
        if _HIP is None:   # the HIP runtime torch loaded (same soname as the library's)
            _HIP = ctypes.CDLL("libamdhip64.so.7")
        self.h = ctypes.c_void_p()
        self.stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        self._check(_HIP.hipEventCreateWithFlags(ctypes.byref(self.h),
                                                 ctypes.c_uint(self.DISABLE_SYSTEM_FENCE)))

    @staticmethod
    def _check(rc):
        if rc != 0:
            raise RuntimeError(f"HIP event call failed with error {rc}")

    def record(self):
        self._check(_HIP.hipEventRecord(self.h, self.stream))

    def elapsed_time(self, end: "TimingEvent") -> float:
        ms = ctypes.c_float()
        self._check(_HIP.hipEventElapsedTime(ctypes.byref(ms), self.h, end.h))
        return ms.value

    def __del__(self):
        if _HIP is not None and self.h:
            _HIP.hipEventDestroy(self.h)


def timed_frames(steps: int) -> list:
    """Orbit frames of the timed steps: the fixed window, cycled."""
    return [TIMED_FIRST + k % TIMED_PERIOD for k in range(steps)]


def event_steps(steps: int) -> list:
    """Timed steps that carry timing events: every EVENT_EVERY-th from step
    0, the sample shifted by one window position each pass through the
    window, so that a long run times the render on every frame of it."""
    sampled = list(range(0, steps, EVENT_EVERY))
    if TIMED_PERIOD % EVENT_EVERY == 0:
        sampled = [k + (k // TIMED_PERIOD) % EVENT_EVERY for k in sampled]
    return [k for k in sampled if k < steps]


def warm_frames(warmup: int) -> list:
    """The warmup frames just before the timed window (cycling below it when
    there are more of them than frames before it)."""
    return [TIMED_FIRST - 1 - ((warmup - 1 - k) % TIMED_FIRST) for k in range(warmup)]


def volume_description(w, dtype: str, layout: str) -> str:
    """What the synthetic input of workload w is, in words."""
    v = w.volume
    s = (f"synthetic: seeded {v.octaves}-octave value-noise FBM density {v.n}^3, coverage "
         f"{v.coverage}" + (", slab height profile" if v.height_falloff else ""))
    if w.detail_n:
        s += f", eroded by a {w.detail_n}^3 Worley/value detail volume"
    views = f", {w.views} views" if w.views > 1 else ""
    return s + f"; {dtype} storage, {layout} layout; orbiting camera{views}"


def counter_config(workload: str, dtype: str, layout: str, occupancy: bool) -> dict:
    """The key a counter record is filed under: the render configuration."""
    return {"workload": workload, "dtype": dtype, "layout": layout, "occupancy": occupancy}


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle as it stands, over row bands, all host cores
# ---------------------------------------------------------------------------

def _oracle_band(args):
    name, dtype, frame, y0, y1 = args
    import numpy as np
    from oracle import cloud as O
    from paper_1609_05344_amd import scenes
    w = scenes.workload(name)
    sc = scenes.make_scene(w, dtype=dtype)
    vol = O.OracleVolume(base=sc.base_f64, detail=sc.detail_f64,
                         detail_weight=w.params.detail_weight, detail_tiling=w.params.detail_tiling)
    ys, xs = np.meshgrid(np.arange(y0, y1), np.arange(w.width), indexing="ij")
    pix = np.stack([xs.reshape(-1), ys.reshape(-1)], 1)
    t = time.perf_counter()
    _, lk = O.render(vol, w.camera(frame), w.params, w.width, w.height, frame=frame, pixels=pix,
                     return_lookups=True)
    return lk, time.perf_counter() - t


def cpu_baseline(name: str, dtype: str, frames: int, cores: int) -> dict:
    from paper_1609_05344_amd import scenes
    w = scenes.workload(name)
    scenes.make_scene(w, dtype=dtype)          # generate/cache the volume once
    bands = cores * 4
    edges = [round(i * w.height / bands) for i in range(bands + 1)]
    jobs = [(name, dtype, f, edges[b], edges[b + 1]) for f in range(frames) for b in range(bands)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_band, jobs[:cores])     # warm the workers (imports, volume load)
        t = time.perf_counter()
        res = pool.map(_oracle_band, jobs)
        dt = time.perf_counter() - t
    lookups = sum(r[0] for r in res)
    return {"value": round(lookups / dt / 1e9, 6), "unit": "Gsamples/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{frames} full {w.width}x{w.height} frames of the same workload "
                      f"({lookups} executed lookups, {dt:.1f} s wall), FP64 numpy, "
                      f"{cores} processes over row bands",
            "ms_per_frame": round(dt * 1e3 / frames, 1)}


_SUBSET_SCENES = {}


def _oracle_subset_job(args):
    name, dtype, view, steps, jitter, pix = args
    from dataclasses import replace
    from oracle import cloud as O
    from paper_1609_05344_amd import scenes
    w = scenes.workload(name)
    if (name, dtype) not in _SUBSET_SCENES:     # one volume load per worker process
        sc = scenes.make_scene(w, dtype=dtype)
        _SUBSET_SCENES[(name, dtype)] = O.OracleVolume(
            base=sc.base_f64, detail=sc.detail_f64, detail_weight=w.params.detail_weight,
            detail_tiling=w.params.detail_tiling)
    vol = _SUBSET_SCENES[(name, dtype)]
    p = replace(w.params, steps=steps, jitter=jitter)
    t = time.perf_counter()
    _, lk = O.render(vol, w.camera(0, view=view), p, w.width, w.height, frame=0, pixels=pix,
                     return_lookups=True)
    return lk, time.perf_counter() - t


def oracle_subset(name: str, dtype: str, steps: int, jitter: int, per_view: int,
                  cores: int) -> dict:
    """The oracle's rate on a seeded subset of per_view pixels of every view,
    for a reference too large to render whole on the host (C5 at 128 steps is
    about 59 G lookups a launch). Times the renders only, not volume loads."""
    import numpy as np
    from paper_1609_05344_amd import scenes
    w = scenes.workload(name)
    scenes.make_scene(w, dtype=dtype)          # generate/cache the volume once
    chunks = max(1, 2 * cores // w.views)
    jobs = [(name, dtype, v, steps, jitter, c)
            for v in range(w.views)
            for c in np.array_split(scenes.random_pixels(w.width, w.height, per_view,
                                                         seed=4096 + v), chunks)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_subset_job, [(name, dtype, 0, 1, 0, jobs[0][5][:4])] * cores)  # load
        t = time.perf_counter()
        res = pool.map(_oracle_subset_job, jobs)
        wall = time.perf_counter() - t
    lookups = sum(r[0] for r in res)
    n_pix = per_view * w.views
    full_px = w.width * w.height * w.views
    return {"metric": "oracle rate on a pixel subset", "workload": name, "dtype": dtype,
            "steps": steps, "jitter": JITTER_NAMES[jitter], "pixels": n_pix,
            "views": w.views, "lookups": int(lookups), "wall_s": round(wall, 2),
            "gsamples_per_s": round(lookups / wall / 1e9, 4),
            "ms_per_pixel": round(wall * 1e3 / n_pix, 5),
            "projected_s_per_launch": round(wall / n_pix * full_px, 1),
            "cores": cores, "kind": "oracle",
            "note": "FP64 numpy over the decoded volume, processes over pixel chunks"}


# VALU lane operations the method itself needs (a minimal implementation's
# instruction slots; the op-by-op listing is in the design notes): per
# executed trilinear lookup of the base volume, per primary sample taken, per
# sample that runs the light march, per pixel, and per pixel whose ray hits
# the volume's box.
OPS_PER_LOOKUP = 35
OPS_PER_PRIMARY = 20
OPS_PER_LIT = 22
OPS_PER_PIXEL = 68
OPS_PER_HIT = 15


def algorithmic_ops(cf, torch, np, w, vol, p, frames) -> dict:
    """Units of work per frame (mean over the frames, which may repeat):
    executed lookups, primary samples, lit samples, pixels and hit pixels,
    from the library's lookup trace (outside the timed launches), and the
    lane operations they need."""
    if p.steps > 32 or w.detail_n:
        return None
    V, W, H = w.views, w.width, w.height
    per_frame = {}
    for f in sorted(set(frames)):
        tr = cf.cloud_lookup_trace(vol, [w.camera(f, view=v) for v in range(V)], p, f, W, H)
        t = tr.cpu().numpy().view(np.uint32).reshape(-1, 2)
        m = t[:, 1].astype(np.uint64)
        per_frame[f] = (int(t[:, 0].astype(np.int64).sum()),
                        int(sum(((m >> np.uint64(k)) & np.uint64(1)).sum() for k in range(32))),
                        int((t[:, 0] > 0).sum()))
    frames = list(frames)
    prim = sum(per_frame[f][0] for f in frames)
    lit = sum(per_frame[f][1] for f in frames)
    hit = sum(per_frame[f][2] for f in frames)
    n = len(frames)
    units = {"lookups": (prim + p.light_steps * lit) / n, "primary_samples": prim / n,
             "lit_samples": lit / n, "pixels": V * W * H, "hit_pixels": hit / n}
    ops = (OPS_PER_LOOKUP * units["lookups"] + OPS_PER_PRIMARY * units["primary_samples"]
           + OPS_PER_LIT * units["lit_samples"] + OPS_PER_PIXEL * units["pixels"]
           + OPS_PER_HIT * units["hit_pixels"])
    return {"units_per_launch": {k: round(v) for k, v in units.items()},
            "ops_per_unit": {"lookup": OPS_PER_LOOKUP, "primary_sample": OPS_PER_PRIMARY,
                             "lit_sample": OPS_PER_LIT, "pixel": OPS_PER_PIXEL,
                             "hit_pixel": OPS_PER_HIT},
            "ops_per_launch": round(ops)}


def roofline(rec: dict, alg: dict, render_ms: float, lk_frame: float, bytes_per_lookup: int):
    """The render kernel against the VALU issue peak (the bound: every lookup
    is an 8-texel gather plus about 35 lane operations, and the issue slots
    run about 80 % busy), with the HBM and issued-VALU figures measured by
    rocprofv3 beside it."""
    sec = render_ms * 1e-3
    line = {"bound": "alu", "kernel": "render_kernel", "kernel_ms": round(render_ms, 4),
            "unit": "TOP/s", "peak": round(MI355X_VALU_LANE_INSTR_PER_S / 1e12, 2),
            "peak_note": "VALU lane operations: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz "
                         "(one FP32 op per lane per cycle; packed FP32 is not used)",
            "events": "HIP events on the launch stream, hipEventDisableSystemFence"}
    if alg:
        a = alg["ops_per_launch"] / sec / 1e12
        line.update({"achieved": round(a, 3), "frac": round(a / line["peak"], 4), **alg})
    else:
        line.update({"achieved": None, "frac": None,
                     "note": "no lane-operation count for detail volumes or > 32 steps"})
    traffic = rec.get("traffic_bytes_per_launch")
    line["traffic"] = traffic
    line["hbm"] = None if not traffic else {
        "bytes_per_launch": traffic, "GBps": round(traffic / sec / 1e9, 1),
        "peak_GBps": MI355X_HBM_GBPS, "frac": round(traffic / sec / 1e9 / MI355X_HBM_GBPS, 4),
        "source": "calibrated rocprofv3 FETCH_SIZE + WRITE_SIZE (profiles/render_traffic.json)"}
    n = rec.get("valu_insts_per_launch")
    line["valu_issued"] = None if not n else {
        "wave_insts_per_launch": n,
        "frac": round(n * 64 / sec / MI355X_VALU_LANE_INSTR_PER_S, 4),
        "source": "rocprofv3 SQ_INSTS_VALU x 64 lanes (profiles/render_traffic.json)"}
    line["cache_gathers"] = {"bytes_per_launch": round(lk_frame * bytes_per_lookup),
                             "bytes_per_lookup": bytes_per_lookup,
                             "GBps": round(lk_frame * bytes_per_lookup / sec / 1e9, 1)}
    return line


# ---------------------------------------------------------------------------
# The paper's timing table (Section 4) on this GPU
# ---------------------------------------------------------------------------

PAPER_ROWS = [
    # (label, workload giving the resolution, steps, jitter, resolve, paper's GTX 1080 ms)
    ("Full, 128 steps", "H", 128, 0, False, 297.7),
    ("Half, 128 steps", "Hh", 128, 0, False, 128.0),
    ("Half, 8 steps", "Hh", 8, 0, False, 2.3),
    ("Half, 8 steps, jitter", "Hh", 8, 1, False, 7.5),
    ("Half, 8 steps, jitter, TAA", "Hh", 8, 1, True, 7.5),
    ("Quarter, 8 steps, jitter, TAA", "Hq", 8, 1, True, 2.4),
]


def paper_table(cf, scenes, torch, np, dtype: str, layout: str, frames=range(10, 40)) -> dict:
    """Each row of the paper's timing table: the cloud render at that
    resolution and step count (H's volume and camera orbit), plus the
    resolve and the up-sample + composite into the 1920x1080 frame where the
    row has them. HIP-event means over the frames given, after ten untimed
    frames of the row (the first launch of a kernel in a process is slow);
    lookups counted by the library outside the timed launches."""
    from dataclasses import replace
    base = scenes.workload("H")
    vol = cf.device_volume(scenes.make_scene(base, dtype=dtype), layout=layout, occupancy=True)
    sky = torch.tensor(scenes.sky_background(1920, 1080), device="cuda")
    full = torch.empty((1080, 1920, 4), device="cuda")
    rows = []
    for label, wname, steps, jit, taa, paper_ms in PAPER_ROWS:
        w = scenes.workload(wname)
        W, H = w.width, w.height
        p = replace(base.params, steps=steps, jitter=jit)
        cur = torch.empty((H, W, 4), device="cuda")
        hist = torch.zeros((H, W, 4), device="cuda")
        lk = torch.zeros((1,), dtype=torch.int64, device="cuda")
        for f in frames:
            cf.cloud_count_lookups(vol, base.camera(f), p, f, W, H, out=lk)
        n_lk = int(lk.item()) / len(frames)
        def frame(f, e):
            e[0].record()
            cf.cloud_render(vol, base.camera(f), p, f, W, H, out=cur)
            e[1].record()
            if taa:
                cf.cloud_taa_resolve(cur, hist, hist, w.taa_blend, f)
            e[2].record()
            if (W, H) != (1920, 1080):
                cf.cloud_composite(hist if taa else cur, sky, out=full)
            e[3].record()

        for f in range(max(frames[0] - 10, 0), frames[0]):
            frame(f, [TimingEvent() for _ in range(4)])
        torch.cuda.synchronize()
        ev = [[TimingEvent() for _ in range(4)] for _ in frames]
        for f, e in zip(frames, ev):
            frame(f, e)
        torch.cuda.synchronize()
        r = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
        t = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
        c = float(np.mean([e[2].elapsed_time(e[3]) for e in ev]))
        piped = None
        if taa:
            # the same frames with frame f's render and frame f - 1's resolve
            # in one launch (then the composite of frame f - 1)
            bufs = [cur, torch.empty_like(cur)]
            hist.zero_()
            seq = list(range(max(frames[0] - 10, 0), frames[0])) + list(frames)
            pev = []
            for k, f in enumerate(seq):
                e = [TimingEvent(), TimingEvent()] if f in frames else None
                if e:
                    e[0].record()
                if k == 0:
                    cf.cloud_render(vol, base.camera(f), p, f, W, H, out=bufs[0])
                else:
                    cf.cloud_render_resolve(vol, base.camera(f), p, f, W, H, bufs[(k - 1) & 1], hist,
                                            hist, w.taa_blend, seq[k - 1], out=bufs[k & 1])
                    if (W, H) != (1920, 1080):
                        cf.cloud_composite(hist, sky, out=full)
                if e:
                    e[1].record()
                    pev.append(e)
            torch.cuda.synchronize()
            piped = round(float(np.mean([e[0].elapsed_time(e[1]) for e in pev])), 4)
        rows.append({"row": label, "width": W, "height": H, "render_ms": round(r, 4),
                     "resolve_ms": round(t, 4) if taa else None,
                     "composite_ms": round(c, 4) if (W, H) != (1920, 1080) else None,
                     "total_ms": round(r + (t if taa else 0) + (c if (W, H) != (1920, 1080) else 0), 4),
                     "pipelined_total_ms": piped,
                     "lookups_per_frame": round(n_lk),
                     "gsamples_per_s": round(n_lk / (r * 1e-3) / 1e9, 1),
                     "paper_gtx1080_ms": paper_ms})
    return {"metric": "the paper's timing table (Section 4) on MI355X", "unit": "ms",
            "storage": f"{dtype} {layout}, occupancy skip", "frames": len(frames), "rows": rows}


# ---------------------------------------------------------------------------
# Offset replay: the render's own fetches from precomputed corners
# ---------------------------------------------------------------------------

def pipelined_leg(cf, torch, np, w, vol, p, settle, warm, timed, lk_timed, seq_hist,
                  seq_ms, sky=None, frame_out=None) -> dict:
    """The same frames through cloud_render_resolve: each launch renders frame
    f and resolves frame f - 1 (rendered by the launch before), so a step is
    still one render and one resolve (and, for a display workload, the
    composite of the resolved frame f - 1). The resolved history after the
    same frame sequence is compared bit for bit with the sequential run's."""
    # the measurement legs before this one leave large host arrays behind
    # (lookup traces): collect them now, not in a pause inside the timed loop
    gc.collect()
    W, H, V = w.width, w.height, w.views
    shape = (V, H, W, 4) if V > 1 else (H, W, 4)
    cur = [torch.empty(shape, device=vol.base.device) for _ in range(2)]
    hist = torch.zeros(shape, device=vol.base.device)
    state = {"k": 0, "prev": None}

    def cams(f):
        return [w.camera(f, view=v) for v in range(V)] if V > 1 else w.camera(f)

    def step(f):
        k = state["k"]
        if state["prev"] is None:
            if V > 1:
                cf.cloud_render_views(vol, cams(f), p, f, W, H, out=cur[k & 1])
            else:
                cf.cloud_render(vol, cams(f), p, f, W, H, out=cur[k & 1])
        else:
            cf.cloud_render_resolve(vol, cams(f), p, f, W, H, cur[(k - 1) & 1], hist, hist,
                                    w.taa_blend, state["prev"], out=cur[k & 1])
            if sky is not None:
                cf.cloud_composite(hist, sky, out=frame_out)   # frame f - 1 into the display
        state["prev"], state["k"] = f, k + 1

    for f in warm_frames(settle) + warm:
        step(f)
    torch.cuda.synchronize()
    a, b = TimingEvent(), TimingEvent()
    t0 = time.perf_counter()
    a.record()
    for f in timed:
        step(f)
    b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the last frame's resolve, outside the timed region (the first timed
    # launch resolved the last warm-up frame instead)
    last = cur[(state["k"] - 1) & 1]
    for v in range(V):
        cf.cloud_taa_resolve(last[v] if V > 1 else last, hist[v] if V > 1 else hist,
                             hist[v] if V > 1 else hist, w.taa_blend, state["prev"])
    torch.cuda.synchronize()
    ms = wall * 1e3 / len(timed)
    return {"form": "cloud_render_resolve: the render of frame f and the resolve of frame f - 1 "
                    "in one launch, the resolve's workgroups after the render's",
            "ms_per_step": round(ms, 4),
            "value": round(lk_timed / wall / 1e9, 3),
            "event_ms_per_step": round(a.elapsed_time(b) / len(timed), 4),
            "speedup_vs_sequential": round(seq_ms / ms, 3),
            "history_bitwise_equal": bool(torch.equal(hist, seq_hist))}


def offset_replay(cf, torch, np, w, vol, p, frames):
    """Times cloud_gather_replay on the given frames' recorded lookups (corner
    codes written by cloud_gather_record outside the timed launches): mode 0
    fetches the render's footprints in its per-wavefront order with none of
    its arithmetic, at each residency cap, mode 1 as many uniformly random
    footprints. Reported beside the render's own time on the same frames."""
    if p.steps > 32 or w.detail_n:
        return None
    V, W, H = w.views, w.width, w.height
    frames = list(frames)
    recs = []
    for f in frames:
        cams = [w.camera(f, view=v) for v in range(V)]
        tr = cf.cloud_lookup_trace(vol, cams, p, f, W, H)
        recs.append(cf.cloud_gather_record(vol, cams, p, f, W, H, tr))
        del tr
    out = torch.empty((cf.gather_waves(V, W, H), 64), dtype=torch.int32, device="cuda")

    def timed(mode, bpc, reps):
        for codes, cnt in recs[:2]:
            cf.cloud_gather_replay(vol, V, W, H, codes, cnt, mode=mode, blocks_per_cu=bpc, out=out)
        torch.cuda.synchronize()
        ev = []
        for r in range(reps):
            codes, cnt = recs[r % len(recs)]
            a, b = TimingEvent(), TimingEvent()
            a.record()
            cf.cloud_gather_replay(vol, V, W, H, codes, cnt, mode=mode, blocks_per_cu=bpc, out=out)
            b.record()
            ev.append((a, b))
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ev]))

    by_cap = {bpc: timed(0, bpc, 3 * len(recs)) for bpc in (0, 2, 3, 4, 6)}
    best = min(by_cap, key=by_cap.get)
    rand = timed(1, best, len(recs))
    del recs
    img = torch.empty((V, H, W, 4), device="cuda")
    ev = []
    for r in range(3 * len(frames) + 2):
        f = frames[r % len(frames)]
        a, b = TimingEvent(), TimingEvent()
        a.record()
        cf.cloud_render_views(vol, [w.camera(f, view=v) for v in range(V)], p, f, W, H, out=img)
        b.record()
        ev.append((a, b))
    torch.cuda.synchronize()
    render_ms = float(np.median([a.elapsed_time(b) for a, b in ev[2:]]))
    del img
    return {"kernel": "gather_replay_kernel", "frames": len(frames),
            "replay_ms_by_blocks_per_cu": {str(k): round(v, 4) for k, v in by_cap.items()},
            "replay_ms": round(by_cap[best], 4), "random_ms": round(rand, 4),
            "render_ms": round(render_ms, 4),
            "render_over_replay": round(render_ms / by_cap[best], 4),
            "note": "the replay reads 4 B of recorded corner per lane and lookup instead of "
                    "computing it; it is not a ceiling: the render issues the same fetches faster"}


# ---------------------------------------------------------------------------
# Served form: many camera streams through cloud_serve_* (closed loop)
# ---------------------------------------------------------------------------

def stream_camera(scenes, w, s: int, n_streams: int, f: int):
    """Camera of stream s at its frame f. A multi-view workload gives stream s
    view s (mod the view count); otherwise the streams sit at their own points
    of the orbit, spread evenly around it, so that no two streams render the
    same view, and each advances one degree a frame over the timed window's
    20 degrees."""
    if w.views > 1:
        return w.camera(TIMED_FIRST + f % TIMED_PERIOD, view=s % w.views)
    az = w.azimuth0_deg + TIMED_FIRST + f % TIMED_PERIOD + 360.0 * s / n_streams
    return scenes.orbit_camera(w.radius, az, w.elevation_deg)


def plain_on_stream_cameras(cf, scenes, torch, np, w, vol, p, n_streams: int, rounds: int = 3):
    """The plain single-frame path (cloud_render + cloud_taa_resolve, one frame
    per launch) on the served leg's cameras, the streams taken in turn: its
    frames/s, for the served form's speed-up on the same views."""
    W, H = w.width, w.height
    cur = torch.empty((H, W, 4), device="cuda")
    hist = torch.zeros((H, W, 4), device="cuda")
    seq = [(s, f) for f in range(rounds) for s in range(n_streams)]

    def frame(s, f):
        cf.cloud_render(vol, stream_camera(scenes, w, s, n_streams, f), p, TIMED_FIRST + f, W, H,
                        out=cur)
        cf.cloud_taa_resolve(cur, hist, hist, w.taa_blend, TIMED_FIRST + f)

    for s, f in seq[:n_streams]:
        frame(s, f)
    torch.cuda.synchronize()
    a, b = TimingEvent(), TimingEvent()
    a.record()
    for s, f in seq:
        frame(s, f)
    b.record()
    torch.cuda.synchronize()
    return round(len(seq) * 1e3 / a.elapsed_time(b), 1)


def served_closed_loop(cf, scenes, torch, w, dtype: str, layout: str, n_streams: int,
                       seconds: float, warm_s: float = 0.5, queues: int = 1,
                       graphs: bool = True, window: int = 1, history_in_output: bool = True,
                       start_lead_us: int = 0, plain_same_views: bool = False) -> dict:
    """n_streams streams of the workload, each keeping `window` frames in
    flight: it submits its next frame as soon as one completes. Frames/s and
    frame latency (submit -> done) over the measured window. A multi-view
    workload gives stream s the camera of view s (mod the view count).
    graphs=False makes the server launch its kernels one by one instead of
    replaying captured graphs; history_in_output has each stream resolve
    against its previous frame's output (one output buffer a stream, resolved
    in place) instead of a library copy of the history. plain_same_views also
    times the plain single-frame path on the same volume and cameras."""
    import numpy as np
    sc = scenes.make_scene(w, dtype=dtype)
    vol = cf.device_volume(sc, layout=layout, occupancy=True)
    W, H = w.width, w.height
    plain = (plain_on_stream_cameras(cf, scenes, torch, np, w, vol, w.params, n_streams)
             if plain_same_views else None)
    outs = [torch.empty((H, W, 4), device="cuda") for _ in range(n_streams)]
    frame = [0] * n_streams
    lat, done_t = [], []

    def camera(s, f):
        return stream_camera(scenes, w, s, n_streams, f)

    with cf.Server(vol, budget_bytes=n_streams * W * H * 40, max_batch=64, queues=queues,
                   use_graphs=graphs, history_in_output=history_in_output,
                   start_lead_us=start_lead_us) as srv:
        t_start = time.monotonic()
        for s in range(n_streams):
            for _ in range(window):
                srv.submit(s, camera(s, frame[s]), w.params, W, H, frame[s], outs[s])
                frame[s] += 1
        t_end = t_start + warm_s + seconds
        while time.monotonic() < t_end:
            got = srv.poll(256)
            if not got:
                srv.wait(0.002)
                continue
            for c in got:
                assert c["status"] == 0, c
                s = c["stream_id"]
                if c["t_done_ns"] * 1e-9 >= t_start + warm_s:
                    lat.append((c["t_done_ns"] - c["t_submit_ns"]) * 1e-6)
                    done_t.append(c["t_done_ns"] * 1e-9)
                srv.submit(s, camera(s, frame[s]), w.params, W, H, frame[s], outs[s])
                frame[s] += 1
        st = srv.stats()
    done_t.sort()
    span = done_t[-1] - done_t[0] if len(done_t) > 1 else float("nan")
    fps = (len(done_t) - 1) / span if len(done_t) > 1 else 0.0
    return {"form": f"served, {dtype} storage, {layout} layout", "streams": n_streams,
            "frames_in_flight_per_stream": window,
            "history": "previous output" if history_in_output else "library copy",
            "frames_per_s": round(fps, 1), "ms_per_frame": round(1e3 / fps, 4) if fps else None,
            "latency_p50_ms": round(float(np.percentile(lat, 50)), 3),
            "latency_p99_ms": round(float(np.percentile(lat, 99)), 3),
            "frames": len(lat), "batches": st["batches"],
            "frames_per_batch": round(st["completed"] / max(st["batches"], 1), 2),
            "queues": queues, "graphs": graphs, "start_lead_us": start_lead_us,
            "plain_frames_per_s": plain}


def served_poisson(cf, scenes, torch, rate_hz: float, seconds: float, warm_s: float = 1.0,
                   n_streams: int = 64, seed: int = 5344, ring: int = 4,
                   budget_bytes: int = 64 << 30, queues: int = 1,
                   start_lead_us: int = 0) -> dict:
    """Open-loop serving load: n_streams camera streams, each with a
    resolution from {640x360, 1280x720, 1920x1080, 3840x2160} and a step
    count from {8, 16, 32, 128} drawn once; Poisson arrivals at rate_hz in
    total, each for a uniformly chosen stream; a shared FP16 256^3 volume.
    Each stream renders into a ring of output buffers and resolves against
    its previous output. Latency runs from the scheduled arrival to
    completion."""
    import numpy as np
    from dataclasses import replace
    rng = np.random.default_rng(seed)
    sizes = [(640, 360), (1280, 720), (1920, 1080), (3840, 2160)]
    steps = [8, 16, 32, 128]
    spec = [(sizes[rng.integers(4)], steps[rng.integers(4)]) for _ in range(n_streams)]
    w = scenes.workload("C2")
    # oct: the 128-step unjittered requests of this mix march coherently, where
    # one 16-byte fetch per lookup beats the quad layout's two
    vol = cf.device_volume(scenes.make_scene(w, dtype="f16"), layout="oct", occupancy=True)
    bufs = [[torch.empty((h, wd, 4), device="cuda") for _ in range(ring)] for (wd, h), _ in spec]
    free = [list(range(ring)) for _ in range(n_streams)]
    frame = [0] * n_streams
    params = [replace(w.params, steps=st) for _, st in spec]
    inflight = {}
    lat, done_t = [], []
    busy = nobuf = 0
    gaps = rng.exponential(1.0 / rate_hz, size=int(rate_hz * (warm_s + seconds) * 1.5) + 16)
    which = rng.integers(n_streams, size=gaps.size)
    with cf.Server(vol, budget_bytes=budget_bytes, max_batch=64, max_queue=4096,
                   queues=queues, history_in_output=True, start_lead_us=start_lead_us) as srv:
        t0 = time.monotonic()
        t_arr = t0 + np.cumsum(gaps)
        k, t_end = 0, t0 + warm_s + seconds
        while True:
            now = time.monotonic()
            if now >= t_end:
                break
            while k < t_arr.size and t_arr[k] <= now:
                s = int(which[k])
                if free[s]:
                    b = free[s].pop()
                    (wd, h), _ = spec[s]
                    rc, rid = srv.try_submit(s, stream_camera(scenes, w, s, n_streams, frame[s]),
                                             params[s], wd, h, frame[s], bufs[s][b])
                    if rc == 0:
                        inflight[rid] = (s, b, t_arr[k])
                        frame[s] += 1
                    else:
                        free[s].append(b)
                        busy += 1
                else:
                    nobuf += 1
                k += 1
            for c in srv.poll(512):
                s, b, ta = inflight.pop(c["request_id"])
                free[s].append(b)
                if ta >= t0 + warm_s:
                    lat.append(c["t_done_ns"] * 1e-9 - ta)
                    done_t.append(c["t_done_ns"] * 1e-9)
            nxt = t_arr[k] if k < t_arr.size else t_end
            srv.wait(max(0.0, min(nxt - time.monotonic(), 0.002)))
        backlog = len(inflight)
        st = srv.stats()
    offered = float(np.sum((t_arr >= t0 + warm_s) & (t_arr < t_end)))
    lat_ms = np.array(lat) * 1e3
    return {"rate_hz": rate_hz, "seconds": seconds, "offered": int(offered),
            "completed": len(lat), "completed_per_s": round(len(lat) / seconds, 1),
            "latency_p50_ms": round(float(np.percentile(lat_ms, 50)), 2) if lat else None,
            "latency_p99_ms": round(float(np.percentile(lat_ms, 99)), 2) if lat else None,
            "rejected_busy": busy, "dropped_no_buffer": nobuf, "backlog_at_end": backlog,
            "batches": st["batches"], "streams": n_streams}


def quality_report(cf, scenes, torch) -> dict:
    """Reported numbers (the gates live in the tests):
    * precision forms at C3 (1080p, 128^3 base + 32^3 detail, 16 jittered
      steps): max and p99 abs RGBA error over 20000 seeded pixels of the FP32,
      FP16 and BF16 storage paths against the FP64 oracle on the decoded stored
      volume, and of the 16-bit paths against the oracle on the FP32 volume;
      the same against the FP32 source at H (quad layout, occupancy);
    * 8 jittered steps + TAA against the 128-step unjittered render (C2, 720p):
      the same camera after a 16-frame accumulation at a fixed camera, next to
      one 8-step frame with and without jitter."""
    import numpy as np
    from oracle import cloud as O
    out = {}
    w = scenes.workload("C3")
    pix = scenes.random_pixels(w.width, w.height, 20000, seed=99)
    src32 = scenes.make_scene(w, dtype="f32")

    def ovol(sc):
        return O.OracleVolume(base=sc.base_f64, detail=sc.detail_f64,
                              detail_weight=w.params.detail_weight,
                              detail_tiling=w.params.detail_tiling)

    ref32 = O.render(ovol(src32), w.camera(0), w.params, w.width, w.height, frame=0, pixels=pix)
    prec = {}
    for dt in ("f32", "f16", "bf16"):
        sc = scenes.make_scene(w, dtype=dt)
        vol = cf.device_volume(sc, layout="oct")
        img = cf.cloud_render(vol, w.camera(0), w.params, 0, w.width, w.height).cpu().numpy()
        got = img[pix[:, 1], pix[:, 0]].astype(np.float64)
        ref = ref32 if dt == "f32" else O.render(ovol(sc), w.camera(0), w.params, w.width,
                                                  w.height, frame=0, pixels=pix)
        e_dec, e_src = np.abs(got - ref), np.abs(got - ref32)
        prec[dt] = {"max_vs_oracle_on_stored": float(e_dec.max()),
                    "p99_vs_oracle_on_stored": float(np.percentile(e_dec, 99)),
                    "max_vs_oracle_on_f32_source": float(e_src.max()),
                    "p99_vs_oracle_on_f32_source": float(np.percentile(e_src, 99))}
    out["precision_C3"] = prec
    # the headline workload's 16-bit forms (quad layout, occupancy) against the
    # oracle on the FP32 source, orbit frame 400
    wh = scenes.workload("H")
    pixh = scenes.random_pixels(wh.width, wh.height, 20000, seed=98)
    srch = scenes.make_scene(wh, dtype="f32")
    refh = O.render(ovol(srch), wh.camera(400), wh.params, wh.width, wh.height, frame=400,
                    pixels=pixh)
    prec_h = {}
    for dt in ("f32", "f16", "bf16"):
        vol = cf.device_volume(scenes.make_scene(wh, dtype=dt), layout="quad", occupancy=True)
        img = cf.cloud_render(vol, wh.camera(400), wh.params, 400, wh.width,
                              wh.height).cpu().numpy()
        e = np.abs(img[pixh[:, 1], pixh[:, 0]].astype(np.float64) - refh)
        prec_h[dt] = {"max_vs_oracle_on_f32_source": float(e.max()),
                      "p99_vs_oracle_on_f32_source": float(np.percentile(e, 99))}
    out["precision_H"] = prec_h

    w2 = scenes.workload("C2")
    vol = cf.device_volume(scenes.make_scene(w2), layout="quad", occupancy=True)
    W, H = w2.width, w2.height
    cam = w2.camera(0)
    from dataclasses import replace
    ref = cf.cloud_render(vol, cam, replace(w2.params, steps=128, jitter=0), 0, W, H).cpu().numpy()
    cur = torch.empty((H, W, 4), device="cuda")

    def accumulated(mode):
        hist = torch.zeros((H, W, 4), device="cuda")
        for f in range(16):
            cf.cloud_render(vol, cam, replace(w2.params, jitter=mode), f, W, H, out=cur)
            cf.cloud_taa_resolve(cur, hist, hist, w2.taa_blend, f)
        return hist.cpu().numpy()

    def err(a):
        d = np.abs(a.astype(np.float64) - ref)
        return {"mean_abs": float(d.mean()), "p99_abs": float(np.percentile(d, 99)),
                "max_abs": float(d.max())}

    one = cf.cloud_render(vol, cam, w2.params, 15, W, H).cpu().numpy()
    flat = cf.cloud_render(vol, cam, replace(w2.params, jitter=0), 15, W, H).cpu().numpy()
    # the orbiting camera (1 degree per frame): plain against reprojected
    # history, after 16 frames, against the 128-step render at the last camera
    last = w2.camera(15)
    ref_last = cf.cloud_render(vol, last, replace(w2.params, steps=128, jitter=0), 0, W,
                               H).cpu().numpy()
    plain_h = torch.zeros((H, W, 4), device="cuda")
    bufs = [torch.zeros((H, W, 4), device="cuda") for _ in range(2)]
    for f in range(16):
        cf.cloud_render(vol, w2.camera(f), w2.params, f, W, H, out=cur)
        cf.cloud_taa_resolve(cur, plain_h, plain_h, w2.taa_blend, f)
        c2, dep = cf.cloud_render_depth(vol, w2.camera(f), w2.params, f, W, H)
        cf.cloud_taa_resolve_reproject(c2, dep, bufs[(f + 1) % 2], bufs[f % 2], w2.camera(f),
                                       w2.camera(max(f - 1, 0)), w2.taa_blend, f)

    def err_last(a):
        d = np.abs(a.astype(np.float64) - ref_last)
        return {"mean_abs": float(d.mean()), "p99_abs": float(np.percentile(d, 99)),
                "max_abs": float(d.max())}

    out["orbit_16_frames_vs_128_C2"] = {"plain_taa": err_last(plain_h.cpu().numpy()),
                                        "reprojected_taa": err_last(bufs[15 % 2].cpu().numpy()),
                                        "one_frame": err_last(cur.cpu().numpy())}
    out["steps8_vs_128_C2"] = {"jitter_taa_16_frames": err(accumulated(1)),
                              "jitter_one_frame": err(one), "no_jitter": err(flat),
                              "tile_jitter_taa_16_frames": err(accumulated(2)),
                              "frame_jitter_taa_16_frames": err(accumulated(3))}
    return out


# ---------------------------------------------------------------------------
# GPU run
# ---------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=200,
                    help="untimed frames first: the GPU clocks settle over the first ~20 ms of load")
    ap.add_argument("--workload", default="H")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--layout", default="quad", choices=["dense", "quad", "oct"])
    ap.add_argument("--served-streams", type=int, default=0,
                    help="closed-loop streams of the served leg (0: 64, or the view count of a "
                         "multi-view workload)")
    ap.add_argument("--served-seconds", type=float, default=2.0)
    ap.add_argument("--served-dtype", default="f16", choices=["f32", "f16", "bf16"])
    ap.add_argument("--served-layout", default="quad", choices=["dense", "quad", "oct"])
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--paper-table", action="store_true",
                    help="time the rows of the paper's timing table and exit")
    ap.add_argument("--taa", default="plain", choices=["plain", "reproject"],
                    help="temporal resolve: plain (the history as is) or reprojected through "
                         "the previous camera with the render's depth")
    ap.add_argument("--jitter-mode", type=int, default=None, choices=[0, 1, 2, 3],
                    help="start offsets: 0 none, 1 per pixel (the workload's), 2 per 8x8 tile, "
                         "3 per frame")
    ap.add_argument("--no-pipelined", action="store_true",
                    help="skip the pipelined leg (cloud_render_resolve: frame f's render and "
                         "frame f - 1's resolve in one launch)")
    ap.add_argument("--no-replay", action="store_true",
                    help="skip the offset-replay measurement")
    ap.add_argument("--serve-queues", type=int, default=1, choices=[1, 2])
    ap.add_argument("--served-window", type=int, default=0, choices=[0, 1, 2],
                    help="frames each closed-loop stream keeps in flight (0: 2 for fewer than "
                         "16 streams, else 1)")
    ap.add_argument("--served-history", default="output", choices=["output", "library"],
                    help="served streams resolve against their previous output, or against "
                         "a library copy of the history")
    ap.add_argument("--serve-blocks-per-cu", type=int, default=0,
                    help="cap on the persistent serving render's workgroups per CU in the "
                         "closed-loop served leg (0: the server's automatic choice; the "
                         "open-loop mix always runs with it)")
    ap.add_argument("--serve-lead-us", type=int, default=0,
                    help="batch start lead of the server (0: its default; -1: start each "
                         "batch as soon as a slot is free)")
    ap.add_argument("--serve-graphs", type=int, default=1, choices=[0, 1],
                    help="served leg: 1 replays captured graphs, 0 launches kernels one by one")
    ap.add_argument("--no-occupancy", action="store_true",
                    help="render without the exact empty-space-skipping bitmap")
    ap.add_argument("--serve-poisson", default="",
                    help="comma-separated total arrival rates (req/s): run only the open-loop "
                         "64-stream serving load at each rate and print one JSON line")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--no-c4", action="store_true",
                    help="skip the open-loop 64-stream serving leg of the default line")
    ap.add_argument("--c4-seconds", type=float, default=3.0,
                    help="measured seconds per rate of the default line's open-loop leg")
    ap.add_argument("--quality", action="store_true",
                    help="print the precision-form and step-count error report instead")
    ap.add_argument("--cpu-frames", type=int, default=36)
    ap.add_argument("--oracle-ref", default="",
                    help="time the FP64 oracle's 128-step unjittered reference of this workload "
                         "on 4096 seeded pixels per view (CPU only), one JSON line")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="launch one plain copy of this many MiB first (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: there is no multi-GPU path (frames, views "
              "and serving streams are independent, so each GPU would take whole ones)",
              file=sys.stderr)
        sys.exit(2)

    if args.paper_table:
        import numpy as np
        import torch
        import paper_1609_05344_amd as cf
        from paper_1609_05344_amd import scenes
        for dt, lay in (("f32", "quad"), ("f16", "oct")):
            print(json.dumps(paper_table(cf, scenes, torch, np, dt, lay)), flush=True)
        return

    if args.oracle_ref:
        w = args.oracle_ref
        print(json.dumps(oracle_subset(w, "f16" if w == "C5" else "f32", 128, 0, 4096,
                                       min(os.cpu_count() or 1, 16))), flush=True)
        return

    if args.quality:
        import torch
        import paper_1609_05344_amd as cf
        from paper_1609_05344_amd import scenes
        print(json.dumps({"metric": "RGBA error report", "report": quality_report(cf, scenes, torch)}),
              flush=True)
        return

    if args.serve_poisson:
        import torch
        import paper_1609_05344_amd as cf
        from paper_1609_05344_amd import scenes
        runs = [served_poisson(cf, scenes, torch, float(r), args.serve_seconds,
                               queues=args.serve_queues)
                for r in args.serve_poisson.split(",")]
        print(json.dumps({"metric": "served frame latency p50/p99, open-loop Poisson arrivals",
                          "unit": "ms", "config": {"workload": "64 streams, resolutions in "
                          "{640x360,1280x720,1920x1080,3840x2160}, steps in {8,16,32,128}, "
                          "shared f16 256^3 (oct layout, occupancy), TAA per stream"},
                          "runs": runs}), flush=True)
        return

    cpu = None
    if not args.no_cpu_baseline and args.jitter_mode is None:
        cores = min(os.cpu_count() or 1, 16)
        cpu = cpu_baseline(args.workload, args.dtype, args.cpu_frames, cores)

    import numpy as np
    import torch

    import paper_1609_05344_amd as cf
    from paper_1609_05344_amd import scenes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    w = scenes.workload(args.workload)
    sc = scenes.make_scene(w, dtype=args.dtype)
    vol = cf.device_volume(sc, dev, layout=args.layout, occupancy=not args.no_occupancy)
    W, H, p = w.width, w.height, w.params
    if args.jitter_mode is not None:
        from dataclasses import replace
        p = replace(p, jitter=args.jitter_mode)

    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib * (1 << 20) // 4
        a = torch.ones(n, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # The timed window is fixed whatever --warmup is: timed step k renders
    # orbit frame TIMED_FIRST + (k mod TIMED_PERIOD), and the warm-up frames
    # are the ones just before it. Executed lookups per frame come from the
    # library's counter, outside the timed region.
    timed = timed_frames(args.steps)
    warm = warm_frames(args.warmup)
    counts = torch.zeros((TIMED_PERIOD,), dtype=torch.int64, device=dev)
    for k in range(TIMED_PERIOD):
        for v in range(w.views):
            cf.cloud_count_lookups(vol, w.camera(TIMED_FIRST + k, view=v), p, TIMED_FIRST + k, W, H,
                                   out=counts[k:k + 1])
    counts = counts.cpu().numpy()

    V = w.views
    cur = torch.empty((V, H, W, 4), device=dev)
    hist = torch.zeros((V, H, W, 4), device=dev)
    reproject = args.taa == "reproject"
    if reproject:
        assert V == 1, "the reprojected resolve is measured on single-view workloads"
        depth = torch.empty((H, W), device=dev)
        hist2 = torch.zeros((H, W, 4), device=dev)
    if w.display:
        assert V == 1, "display workloads are single-view"
        DW, DH = w.display
        sky = torch.tensor(scenes.sky_background(DW, DH), device=dev)
        frame_out = torch.empty((DH, DW, 4), device=dev)
    # per sampled timed frame (every EVENT_EVERY-th): before and after the
    # render; the next sampled frame's first event, or `end`, closes its group
    sampled = event_steps(args.steps)
    ev = {k: (TimingEvent(), TimingEvent()) for k in sampled}
    end = TimingEvent()

    def frame(f, events=None):
        resolve(f, events)
        if w.display:
            resolved = hist[0] if not reproject or f % 2 == 1 else hist2
            cf.cloud_composite(resolved, sky, out=frame_out)

    def resolve(f, events=None):
        if events:
            events[0].record()
        if reproject:
            cf.cloud_render_depth(vol, w.camera(f), p, f, W, H, out=cur[0], depth=depth)
            if events:
                events[1].record()
            src, dst = (hist[0], hist2) if f % 2 == 0 else (hist2, hist[0])
            cf.cloud_taa_resolve_reproject(cur[0], depth, src, dst, w.camera(f),
                                           w.camera(max(f - 1, 0)), w.taa_blend, f)
            return
        if V == 1:
            cf.cloud_render(vol, w.camera(f), p, f, W, H, out=cur[0])
        else:
            cf.cloud_render_views(vol, [w.camera(f, view=v) for v in range(V)], p, f, W, H, out=cur)
        if events:
            events[1].record()
        for v in range(V):
            cf.cloud_taa_resolve(cur[v], hist[v], hist[v], w.taa_blend, f)

    # The GPU's clocks settle over the first ~20 ms of load: short warm-ups
    # are topped up with untimed frames of the same cycle, so that every run
    # times the steady state.
    settle = max(0, SETTLE_FRAMES - args.warmup)
    for f in warm_frames(settle) + warm:
        frame(f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, f in enumerate(timed):
        frame(f, ev.get(k))
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    render_ms = float(np.mean([a.elapsed_time(b) for a, b in ev.values()]))
    # mean frame time of each group of EVENT_EVERY frames (the last may be shorter)
    starts = [ev[k][0] for k in sampled] + [end]
    bounds = sampled + [args.steps]
    frame_ms = np.array([starts[i].elapsed_time(starts[i + 1]) / (bounds[i + 1] - bounds[i])
                         for i in range(len(sampled))])
    lk_timed = int(sum(counts[k % TIMED_PERIOD] for k in range(args.steps)))
    lk_frame = lk_timed / args.steps
    ms_per_step = wall * 1e3 / args.steps
    value = lk_timed / wall / 1e9

    elem = 4 if args.dtype == "f32" else 2
    bytes_per_lookup = 8 * elem * (2 if w.detail_n else 1)   # base (+ detail) footprint
    # the roofline's work figures are for the frames whose render was timed
    alg = algorithmic_ops(cf, torch, np, w, vol, p, [timed[k] for k in sampled])
    lk_sampled = float(np.mean([counts[k % TIMED_PERIOD] for k in sampled]))
    traffic_key = counter_config(w.name, args.dtype, args.layout, not args.no_occupancy)
    line = {
        "metric": "Gsamples/s @1080p 8-step+TAA (executed trilinear density lookups per second; "
                  "ms/frame in ms_per_step)",
        "value": round(value, 3),
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle_frames": max(0, SETTLE_FRAMES - args.warmup),
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": PATH_DTYPE[args.dtype],
        "data": volume_description(w, args.dtype, args.layout),
        "config": {"workload": f"{w.name}: {w.description}", "width": W, "height": H,
                   "display": list(w.display) or None,
                   "primary_steps": p.steps, "light_steps": p.light_steps, "jitter": JITTER_NAMES[p.jitter],
                   "integration": "analytic", "taa_blend": w.taa_blend, "taa": args.taa,
                   "volume": f"{w.volume.n}^3 {args.dtype}", "layout": args.layout,
                   "occupancy_skip": not args.no_occupancy,
                   "lookups_per_frame": round(lk_frame),
                   "nominal_lookups_per_frame": V * W * H * p.steps * (1 + p.light_steps)},
        "roofline": roofline(recorded_counters(traffic_key), alg, render_ms, lk_sampled,
                             bytes_per_lookup),
        "cpu_baseline": cpu,
        # HIP-event time per frame over each group of EVENT_EVERY timed
        # frames; the render kernel's time (roofline) is timed on the first
        # frame of each group
        "frame_ms": {"median": round(float(np.median(frame_ms)), 4),
                     "p90": round(float(np.percentile(frame_ms, 90)), 4),
                     "frames_per_group": EVENT_EVERY},
        "render_kernel_timed_frames": len(sampled),
    }
    if not args.no_pipelined and not reproject:
        line["pipelined"] = pipelined_leg(cf, torch, np, w, vol, p, settle, warm, timed, lk_timed,
                                          hist if V > 1 else hist[0], ms_per_step,
                                          sky if w.display else None,
                                          frame_out if w.display else None)
    if not args.no_replay:
        line["offset_replay"] = offset_replay(cf, torch, np, w, vol, p,
                                              range(TIMED_FIRST, TIMED_FIRST + 4))
    if not args.no_served:
        n_streams = args.served_streams or (64 if w.views == 1 else w.views)
        plain_views = (plain_on_stream_cameras(cf, scenes, torch, np, w, vol, p, n_streams)
                       if w.views == 1 and not w.display else None)
        del cur, hist, vol
        torch.cuda.empty_cache()
        window = args.served_window or (2 if n_streams < 16 else 1)
        cf.cloud_tune("serve_blocks_per_cu", args.serve_blocks_per_cu)
        served = served_closed_loop(cf, scenes, torch, w, args.served_dtype, args.served_layout,
                                    n_streams, args.served_seconds, queues=args.serve_queues,
                                    graphs=args.serve_graphs == 1, window=window,
                                    history_in_output=args.served_history == "output",
                                    start_lead_us=args.serve_lead_us,
                                    plain_same_views=plain_views is not None)
        # the served form against the plain path with the same storage on the
        # same cameras (a multi-view workload: the timed plain step, which
        # renders and resolves every view once); beside it, the plain path
        # with the timed step's storage on those cameras
        if served["plain_frames_per_s"] is not None:
            served["plain_form"] = (f"{args.served_dtype} {args.served_layout}, one frame a launch, "
                                    f"on the same {n_streams} stream cameras")
            served["plain_timed_storage"] = {
                "form": f"{args.dtype} {args.layout}, one frame a launch, same cameras",
                "frames_per_s": plain_views,
                "speedup": round(served["frames_per_s"] / plain_views, 3)}
        else:
            served["plain_frames_per_s"] = round(V * 1e3 / ms_per_step, 1)
            served["plain_form"] = f"the timed plain step ({args.dtype} {args.layout})"
        served["speedup_vs_plain"] = round(served["frames_per_s"] / served["plain_frames_per_s"], 3)
        served["serve_blocks_per_cu"] = args.serve_blocks_per_cu or "auto"
        line["served"] = served
    if not args.no_served and not args.no_c4:
        # the serving form's latency metric: 64 streams of mixed resolutions and
        # step counts, open-loop Poisson arrivals at the specified total rate,
        # and at half of it
        cf.cloud_tune("serve_blocks_per_cu", 0)
        line["served_c4"] = {
            "workload": "64 streams, resolutions in {640x360,1280x720,1920x1080,3840x2160}, "
                        "steps in {8,16,32,128}, shared f16 256^3 (oct layout, occupancy), TAA "
                        "per stream, Poisson arrivals",
            "runs": [served_poisson(cf, scenes, torch, r, args.c4_seconds, warm_s=1.0,
                                    queues=args.serve_queues) for r in (2000.0, 1000.0)]}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Parity of the HIP path with the FP64 oracle, through the C ABI.

Every case runs the library and the oracle on the same seeded inputs and
compares element by element: bit-exact for the jitter hash, max-abs RGBA
<= 1e-4 for float32 volumes and <= 2e-3 for 16-bit volumes (against the
oracle on the exactly decoded volume). Full-size workloads are compared on a
seeded sample of pixels the oracle computes one by one.
"""

import math
import os
import sys
from dataclasses import replace

import numpy as np
import pytest

from oracle import cloud as O
from paper_1609_05344_amd import scenes
from tests.helpers import FP32_TOL, HALF_TOL, const_scene, max_err, oracle_volume, to_np

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cf():
    import torch
    import paper_1609_05344_amd as cf
    assert torch.cuda.is_available()
    cf.load()
    return cf


@pytest.fixture(scope="module")
def torch():
    import torch
    return torch


def params(**kw):
    return replace(scenes.Params(steps=8, light_steps=6, alpha=10.0, g=0.6, jitter=0, t_eps=0.0), **kw)


def run_rays(cf, torch, scene, o, d, p, pixel_xy=None, frame=0):
    vol = cf.device_volume(scene)
    ot = torch.tensor(np.asarray(o, np.float32), device="cuda")
    dt = torch.tensor(np.asarray(d, np.float32), device="cuda")
    pt = None if pixel_xy is None else torch.tensor(np.asarray(pixel_xy, np.uint32).astype(np.int32),
                                                    device="cuda")
    out = cf.cloud_march_rays(vol, ot, dt, pt, p, frame)
    torch.cuda.synchronize()
    return to_np(out).astype(np.float64)


# ---------------------------------------------------------------------------
# jitter hash: bit-exact
# ---------------------------------------------------------------------------

def test_jitter_bits_exact(cf, torch):
    say("jitter bits 256x256 grid")
    py, px = np.meshgrid(np.arange(256), np.arange(256), indexing="ij")
    pts = np.stack([px.reshape(-1), py.reshape(-1)], 1).astype(np.uint32)
    pt = torch.tensor(pts.astype(np.int32), device="cuda")
    for frame in (0, 1, 7, 15, 1 << 31):
        for seed in (0, 1609, 0xFFFFFFFF):
            got = to_np(cf.cloud_jitter_offsets(pt, frame, seed)).astype(np.int64)
            want = np.round(O.jitter_offset(pts[:, 0], pts[:, 1], frame, seed) * 2 ** 24).astype(np.int64)
            assert np.array_equal(got, want), (frame, seed)
    with open(os.path.join(HERE, "golden", "pcg_kat.txt")) as f:
        rows = [l.split() for l in f if l.startswith("jit")]
    pts = np.array([[int(r[1]), int(r[2])] for r in rows], np.uint32)
    for k, r in enumerate(rows):
        got = to_np(cf.cloud_jitter_offsets(torch.tensor(pts[k:k + 1].astype(np.int32), device="cuda"),
                                            int(r[3]), int(r[4])))
        assert int(got[0]) == int(r[5])


# ---------------------------------------------------------------------------
# closed forms through explicit rays (homogeneous box)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("N", [1, 3, 8, 128, 4096])
def test_gpu_homogeneous_closed_forms(cf, torch, N):
    say(f"homogeneous closed forms N={N}")
    c, alpha = 0.4, 8.0
    sc = const_scene(c)
    o = [(0.0, 2.0, 0.0), (-3.0, 0.1, 0.2), (2.0, 1.5, 1.7)]
    d = [(0.0, -1.0, 0.0), (1.0, 0.0, 0.0), (-0.9, -0.7, -0.8)]
    pxy = [(3, 4), (100, 7), (5, 999)]
    tol = FP32_TOL if N == 4096 else 1e-5
    for integ in (0, 1):
        p = params(steps=N, alpha=alpha, integration=integ, sun_color=(0.0, 0.0, 0.0),
                   ambient=(0.2, 0.3, 0.5), jitter=1)
        got = run_rays(cf, torch, sc, o, d, p, pixel_xy=pxy, frame=2)
        oo, dd = np.array(o), np.array(d)
        dd = dd / np.linalg.norm(dd, axis=1, keepdims=True)
        tn, tf, hit = O.ray_box(oo, dd, (-0.5,) * 3, (0.5,) * 3)
        A = -np.expm1(-c * alpha * (tf - tn))
        assert max_err(got[:, 3], A) < tol
        if integ == 1:
            assert max_err(got[:, :3], A[:, None] * np.array([0.2, 0.3, 0.5])[None, :]) < tol
        else:
            x = c * alpha * (tf - tn) / N
            naive = (x * np.exp(-x) * -np.expm1(-N * x) / -np.expm1(-x))[:, None] * np.array([0.2, 0.3, 0.5])
            assert max_err(got[:, :3], naive) < tol


@pytest.mark.parametrize("N,ratio", [(8, 0.58198), (16, 0.77075), (128, 0.96908), (4096, 0.99902)])
def test_gpu_step_dependence_ratio(cf, torch, N, ratio):
    say(f"naive/analytic ratio N={N}")
    sc = const_scene(0.8)
    p = params(steps=N, alpha=10.0, sun_color=(0, 0, 0), ambient=(0.2, 0.2, 0.2))
    a = run_rays(cf, torch, sc, [(0, 2, 0)], [(0, -1, 0)], replace(p, integration=1))[0]
    n = run_rays(cf, torch, sc, [(0, 2, 0)], [(0, -1, 0)], replace(p, integration=0))[0]
    assert abs(a[0] - 0.2 * -math.expm1(-8.0)) < 1e-5          # invariant in N
    assert n[0] / a[0] == pytest.approx(ratio, abs=2e-4)


@pytest.mark.parametrize("N", [1, 2, 8, 128])
def test_gpu_sun_closed_forms(cf, torch, N):
    say(f"front/back lit N={N}")
    c, alpha, H = 0.1, 10.0, 1.0
    sig = c * alpha
    x = sig * H / N
    Cs, a = np.array(scenes.SUN_COLOR), np.array(scenes.AMBIENT)
    p = params(steps=N, alpha=alpha, sun_dir=(0.0, 1.0, 0.0), g=0.6, jitter=1)
    pxy = [(11, 22), (33, 44)]
    j = O.jitter_offset(np.array([11, 33]), np.array([22, 44]), 5, p.seed)
    got = run_rays(cf, torch, const_scene(c), [(0, 2, 0), (0, -2, 0)], [(0, -1, 0), (0, 1, 0)],
                   p, pixel_xy=pxy, frame=5)
    front = Cs * O.hg_phase(-1.0, 0.6) * -math.expm1(-2 * sig * H) * math.exp(-x * j[0]) / (1 + math.exp(-x)) \
        + a * -math.expm1(-sig * H)
    back = Cs * O.hg_phase(1.0, 0.6) * math.exp(-sig * H) * N * -math.expm1(-x) * math.exp(x * j[1]) \
        + a * -math.expm1(-sig * H)
    assert max_err(got[0, :3], front) < 1e-5
    assert max_err(got[1, :3], back) < 1e-5


def test_gpu_empty_and_miss_exact_zero(cf, torch):
    say("empty volume and misses")
    p = params(steps=16, jitter=1)
    out = run_rays(cf, torch, const_scene(0.0), [(0, 2, 0), (3, 3, 3)], [(0, -1, 0), (1, 0, 0)], p,
                   pixel_xy=[(1, 1), (2, 2)])
    assert np.all(out == 0.0)
    vol = cf.device_volume(scenes.make_scene(scenes.workload("C1")))
    img = to_np(cf.cloud_render(vol, scenes.orbit_camera(2.0, 210.0, 20.0), p, 0, 64, 64))
    gx, gy = np.meshgrid(np.arange(64), np.arange(64), indexing="xy")
    o, d = O.camera_rays(scenes.orbit_camera(2.0, 210.0, 20.0), 64, 64, gx.reshape(-1), gy.reshape(-1))
    _, _, hit = O.ray_box(o, d, (-0.5,) * 3, (0.5,) * 3)
    assert np.all(img.reshape(-1, 4)[~hit] == 0.0)


def test_gpu_telescoping_on_noise(cf, torch):
    say("telescoping invariant on C2 volume, 320x180")
    w = scenes.workload("C2")
    vol = cf.device_volume(scenes.make_scene(w))
    p = replace(w.params, sun_color=(0.0, 0.0, 0.0), ambient=(0.2, 0.25, 0.3))
    img = to_np(cf.cloud_render(vol, w.camera(0), p, 0, 320, 180)).astype(np.float64)
    a = np.array([0.2, 0.25, 0.3])
    assert max_err(img[..., :3], img[..., 3:4] * a) < 1e-5
    assert img[..., 3].max() > 0.5


# ---------------------------------------------------------------------------
# full frames and sampled pixels against the oracle
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("integ,jit", [(1, 0), (0, 0), (1, 1), (0, 1), (1, 2), (1, 3), (0, 2)])
def test_c1_full_frame(cf, torch, integ, jit):
    say(f"C1 64x64 full frame integ={integ} jitter={jit}")
    w = scenes.workload("C1")
    sc = scenes.make_scene(w)
    p = replace(w.params, integration=integ, jitter=jit)
    got = to_np(cf.cloud_render(cf.device_volume(sc), w.camera(0), p, 3, 64, 64))
    want = O.render(oracle_volume(sc), w.camera(0), p, 64, 64, frame=3)
    assert max_err(got, want) < FP32_TOL
    assert want[..., 3].max() > 0.5


@pytest.mark.parametrize("W,H", [(1, 1), (17, 9), (37, 23), (100, 3), (3, 50)])
def test_ragged_sizes(cf, torch, W, H):
    say(f"ragged {W}x{H}")
    w = scenes.workload("C2")
    sc = scenes.make_scene(w)
    cam = scenes.orbit_camera(1.0, 215.0, 10.0)
    got = to_np(cf.cloud_render(cf.device_volume(sc), cam, w.params, 1, W, H))
    want = O.render(oracle_volume(sc), cam, w.params, W, H, frame=1)
    assert max_err(got, want) < FP32_TOL


@pytest.mark.parametrize("W,H", [(65536, 2), (3, 65536)])
def test_maximum_image_extents_sampled(cf, torch, W, H):
    # the largest width and height the library accepts, on thin images
    say(f"maximum extent {W}x{H}: sampled parity")
    w = scenes.workload("C2")
    sc = scenes.make_scene(w)
    cam = scenes.Camera(pos=(0.0, 0.05, 1.2), target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0),
                        vfov_deg=50.0)
    got = to_np(cf.cloud_render(cf.device_volume(sc, layout="oct", occupancy=True), cam,
                                w.params, 2, W, H))
    pix = scenes.random_pixels(W, H, 1500, seed=W + H)
    ends = np.array([[0, 0], [W - 1, 0], [0, H - 1], [W - 1, H - 1]])
    # with so extreme an aspect only the rays next to the centre line meet the
    # volume: take a band around it as well
    band = np.array([[x, y] for x in range(max(W // 2 - 24, 0), min(W // 2 + 24, W))
                     for y in range(max(H // 2 - 24, 0), min(H // 2 + 24, H))])
    pix = np.concatenate([pix, ends, band])
    want = O.render(oracle_volume(sc), cam, w.params, W, H, frame=2, pixels=pix)
    assert max_err(got[pix[:, 1], pix[:, 0]], want) < FP32_TOL
    assert want[:, 3].max() > 0.05


@pytest.mark.parametrize("dims", [(2, 2, 2), (257, 3, 2), (2, 300, 5)])
@pytest.mark.parametrize("layout", ["dense", "quad", "oct"])
def test_degenerate_volume_shapes(cf, torch, dims, layout):
    # the smallest volume and long thin ones, every layout, against the oracle
    say(f"volume {dims} {layout}: full frame vs oracle")
    w = scenes.workload("C1", jitter=1)
    rng = np.random.default_rng(sum(dims))
    nx, ny, nz = dims
    base = np.clip(rng.uniform(-0.3, 1.0, size=(nz, ny, nx)), 0, 1)
    st = scenes.quantise(base, "f32")
    sc = scenes.Scene(w, st, scenes.decode(st, "f32"))
    vol = cf.device_volume(sc, layout=layout, occupancy=layout != "dense")
    cam = scenes.orbit_camera(1.6, 205.0, 30.0)
    got = to_np(cf.cloud_render(vol, cam, w.params, 1, 48, 40))
    want = O.render(oracle_volume(sc), cam, w.params, 48, 40, frame=1)
    assert max_err(got, want) < FP32_TOL
    assert want[..., 3].max() > 0.05


@pytest.mark.parametrize("name,frame", [("C2", 0), ("C2", 9), ("C2ref", 0), ("H", 3)])
def test_full_size_sampled(cf, torch, name, frame):
    w = scenes.workload(name)
    say(f"{name} {w.width}x{w.height} frame {frame}: sampled parity")
    sc = scenes.make_scene(w)
    got = to_np(cf.cloud_render(cf.device_volume(sc), w.camera(frame), w.params, frame, w.width, w.height))
    pix = scenes.random_pixels(w.width, w.height, 3000, seed=frame + 17)
    want = O.render(oracle_volume(sc), w.camera(frame), w.params, w.width, w.height, frame=frame,
                    pixels=pix)
    assert max_err(got[pix[:, 1], pix[:, 0]], want) < FP32_TOL
    # the image edges and corners are part of every sample
    edge = np.array([[0, 0], [w.width - 1, 0], [0, w.height - 1], [w.width - 1, w.height - 1],
                     [w.width // 2, w.height // 2]])
    want_e = O.render(oracle_volume(sc), w.camera(frame), w.params, w.width, w.height, frame=frame,
                      pixels=edge)
    assert max_err(got[edge[:, 1], edge[:, 0]], want_e) < FP32_TOL


@pytest.mark.parametrize("jit", [2, 3])
def test_coherent_jitter_sampled_and_structured(cf, torch, jit):
    w = scenes.workload("H")
    say(f"H 1080p jitter mode {jit}: sampled parity, explicit rays")
    sc = scenes.make_scene(w)
    p = replace(w.params, jitter=jit)
    vol = cf.device_volume(sc, layout="quad", occupancy=True)
    got = to_np(cf.cloud_render(vol, w.camera(4), p, 4, w.width, w.height))
    pix = scenes.random_pixels(w.width, w.height, 2000, seed=41 + jit)
    want = O.render(oracle_volume(sc), w.camera(4), p, w.width, w.height, frame=4, pixels=pix)
    assert max_err(got[pix[:, 1], pix[:, 0]], want) < FP32_TOL
    # explicit rays with pixel coordinates take the same mode
    o, d = O.camera_rays(w.camera(4), w.width, w.height, pix[:, 0], pix[:, 1])
    dev = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    rays = to_np(cf.cloud_march_rays(vol, dev(o, torch.float32), dev(d, torch.float32),
                                     dev(pix.astype(np.int32), torch.int32), p, 4))
    assert max_err(rays, want) < FP32_TOL


def test_views_match_single_renders(cf, torch):
    say("multi-view launch vs single renders (18 views, chunked)")
    w = scenes.workload("C2")
    vol = cf.device_volume(scenes.make_scene(w))
    cams = [scenes.orbit_camera(1.0, 210.0 + 20 * v, 10.0) for v in range(18)]
    multi = to_np(cf.cloud_render_views(vol, cams, w.params, 4, 48, 40))
    for v in (0, 5, 16, 17):
        single = to_np(cf.cloud_render(vol, cams[v], w.params, 4, 48, 40))
        assert np.array_equal(multi[v], single)


@pytest.mark.parametrize("frame", [3, 4])
@pytest.mark.parametrize("shape", [(1920, 1080, 1), (333, 77, 1), (200, 120, 5)])
def test_tile_walks_render_identically(cf, torch, shape, frame):
    # the block -> tile walk (super-tile size, XCD interleave, and its mirror
    # on odd frames) only reorders work: every walk must write every pixel
    # once, with the same values
    W, H, views = shape
    say(f"tile walks: {views} x {W}x{H}, frame {frame}, every setting bitwise equal to row-major")
    w = scenes.workload("H")
    vol = cf.device_volume(scenes.make_scene(w, dtype="f16"), layout="oct", occupancy=True)
    cams = [w.camera(frame + v) for v in range(views)]
    results = {}
    try:
        for S, inter in ((0, 0), (-1, -1), (0, 16), (3, 7), (4, 16), (8, 64), (8, 0), (5, 1), (64, 4096)):
            cf.cloud_tune("supertile", S)
            cf.cloud_tune("xcd_run", inter)
            out = torch.full((views, H, W, 4), float("nan"), device="cuda")
            results[(S, inter)] = to_np(cf.cloud_render_views(vol, cams, w.params, frame, W, H,
                                                              out=out))
    finally:
        cf.cloud_tune("supertile", -1)
        cf.cloud_tune("xcd_run", -1)
    ref = results[(0, 0)]
    assert not np.isnan(ref).any()
    assert ref[..., 3].max() > 0.3
    for k, v in results.items():
        assert np.array_equal(v, ref), k


def test_deterministic(cf, torch):
    say("determinism")
    w = scenes.workload("H")
    vol = cf.device_volume(scenes.make_scene(w))
    a = to_np(cf.cloud_render(vol, w.camera(2), w.params, 2, w.width, w.height))
    b = to_np(cf.cloud_render(vol, w.camera(2), w.params, 2, w.width, w.height))
    assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# 16-bit storage
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_half_storage_small_full_frame(cf, torch, dtype):
    say(f"C1 {dtype} full frame")
    w = scenes.workload("C1")
    sc = scenes.make_scene(w, dtype=dtype)
    got = to_np(cf.cloud_render(cf.device_volume(sc), w.camera(0), w.params, 0, 64, 64))
    want = O.render(oracle_volume(sc), w.camera(0), w.params, 64, 64)
    assert max_err(got, want) < HALF_TOL


@pytest.mark.parametrize("dtype", ["f16", "bf16", "f32"])
def test_c3_detail_sampled(cf, torch, dtype):
    w = scenes.workload("C3")
    say(f"C3 {dtype} {w.width}x{w.height} with detail erosion: sampled parity")
    sc = scenes.make_scene(w, dtype=dtype)
    got = to_np(cf.cloud_render(cf.device_volume(sc), w.camera(0), w.params, 0, w.width, w.height))
    pix = scenes.random_pixels(w.width, w.height, 2000, seed=33)
    want = O.render(oracle_volume(sc), w.camera(0), w.params, w.width, w.height, pixels=pix)
    tol = FP32_TOL if dtype == "f32" else HALF_TOL
    assert max_err(got[pix[:, 1], pix[:, 0]], want) < tol


# ---------------------------------------------------------------------------
# temporal resolve
# ---------------------------------------------------------------------------

# 4096x2050 is past the size at which the resolve's tiles stop being dealt to
# the XCDs in contiguous runs
@pytest.mark.parametrize("W,H", [(1280, 720), (37, 23), (1, 1), (16, 1), (4096, 2050)])
def test_taa_parity(cf, torch, W, H):
    say(f"resolve {W}x{H}")
    rng = np.random.default_rng(W * 7 + H)
    cur = rng.uniform(0, 1, (H, W, 4)).astype(np.float32)
    hist = rng.uniform(-0.2, 1.2, (H, W, 4)).astype(np.float32)
    ct, ht = torch.tensor(cur, device="cuda"), torch.tensor(hist, device="cuda")
    for frame, blend in ((1, 0.1), (5, 1.0), (0, 0.1)):
        out = to_np(cf.cloud_taa_resolve(ct, ht, None, blend, frame))
        want = O.taa_resolve(cur, hist, blend, frame)
        assert max_err(out, want) < 1e-6
    out = to_np(cf.cloud_taa_resolve(ct, None, None, 0.1, 4))
    assert np.array_equal(out, cur)
    # in place: out == history
    h2 = ht.clone()
    cf.cloud_taa_resolve(ct, h2, h2, 0.1, 2)
    assert max_err(to_np(h2), O.taa_resolve(cur, hist, 0.1, 2)) < 1e-6


def test_sequence_render_and_resolve(cf, torch):
    say("C2 volume 160x90, 16-frame orbit, render + resolve chain")
    w = scenes.workload("C2")
    sc = scenes.make_scene(w)
    vol, ovol = cf.device_volume(sc), oracle_volume(sc)
    W, H = 160, 90
    hist_g = torch.zeros((H, W, 4), device="cuda")
    cur_g = torch.empty((H, W, 4), device="cuda")
    hist_o = None
    for f in range(16):
        cf.cloud_render(vol, w.camera(f), w.params, f, W, H, out=cur_g)
        cf.cloud_taa_resolve(cur_g, hist_g, hist_g, w.taa_blend, f)
        cur_o = O.render(ovol, w.camera(f), w.params, W, H, frame=f)
        hist_o = O.taa_resolve(cur_o, hist_o, w.taa_blend, f)
        assert max_err(to_np(cur_g), cur_o) < FP32_TOL, f
        assert max_err(to_np(hist_g), hist_o) < FP32_TOL, f


# ---------------------------------------------------------------------------
# argument checks that need device memory
# ---------------------------------------------------------------------------

def test_abi_device_checks(cf, torch):
    say("ABI device-memory checks")
    w = scenes.workload("C1")
    vol = cf.device_volume(scenes.make_scene(w))
    # buffer checks are exercised without launching anything
    big = torch.empty((1 << 22,), dtype=torch.float32, device="cuda")     # 16 MiB, own segment
    assert cf.cloud_check_buffer(big, big.numel() * 4) == 0
    assert cf.cloud_check_buffer(big.data_ptr() + 64, big.numel() * 4 - 64) == 0
    assert cf.cloud_check_buffer(big, 1 << 30) == -1
    assert "allocation" in cf.last_error()
    host = torch.empty((64, 64, 4))
    assert cf.cloud_check_buffer(host, 16) == -1
    assert cf.cloud_check_buffer(None, 16) == -1
    cur = torch.zeros((8, 8, 4), device="cuda")
    with pytest.raises(cf.CloudError):
        cf.cloud_taa_resolve(cur, cur.clone(), cur, 0.1, 1)     # out aliases current
    bad = replace(w.params, g=1.0)
    with pytest.raises(cf.CloudError):
        cf.cloud_render(vol, w.camera(0), bad, 0, 8, 8)
    torch.cuda.synchronize()


def test_c5_views_sampled(cf, torch):
    w = scenes.workload("C5")
    say(f"C5 {w.views} views of {w.width}x{w.height}, 512^3 f16 oct + occupancy: sampled parity per view")
    sc = scenes.make_scene(w, dtype="f16")
    vol = cf.device_volume(sc, layout="oct", occupancy=True)
    cams = [w.camera(2, view=v) for v in range(w.views)]
    img = cf.cloud_render_views(vol, cams, w.params, 2, w.width, w.height)
    ovol = oracle_volume(sc)
    for v in range(w.views):
        pix = scenes.random_pixels(w.width, w.height, 512, seed=100 + v)
        got = to_np(img[v])[pix[:, 1], pix[:, 0]]
        want = O.render(ovol, cams[v], w.params, w.width, w.height, frame=2, pixels=pix)
        assert max_err(got, want) < HALF_TOL, v
    del img
    torch.cuda.empty_cache()

"""Representative depth and the reprojected temporal resolve, through the C
ABI, against the oracle.

Tolerances. The image of cloud_render_depth is cloud_render's, bit for bit.
Depth is compared where the oracle's alpha is clear of the 0.01 switch
between the weighted mean and the chord middle (|alpha - 0.01| > 1e-3), to
1e-3 absolute: the float32 opacity increments carry about 1e-7 absolute
error each, the weighted sum of up to N of them at distances below 4, over
alpha >= 0.01. One reprojected resolve is held to the float32 gate (1e-4): the
projected coordinate carries about 1e-4 pixels of float32 error at these
widths, times a history gradient below 0.5 per pixel. A chain of resolves
feeds that error back through the history with weight 1 - blend per frame, so
the analysis bounds a chain by 1e-4 / blend = 1e-3 where such an error meets
a sharp history edge every frame. On these seeded orbits the chain stays at
the single frame's render error (max-abs 3.6e-5 on the first frame, falling
to about 3e-6 as the history settles), so chains are held to the float32
gate itself, 1e-4 max-abs, and 2e-6 mean-abs.
"""

import sys

import numpy as np
import pytest

from oracle import cloud as O
from paper_1609_05344_amd import scenes
from tests.helpers import FP32_TOL, max_err, oracle_volume, to_np

pytestmark = pytest.mark.gpu


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


def depth_close(got, want, alpha):
    clear = np.abs(alpha - O.DEPTH_ALPHA_MIN) > 1e-3
    assert clear.mean() > 0.95
    return float(np.max(np.abs(got - want)[clear]))


@pytest.mark.parametrize("layout", ["dense", "quad"])
def test_depth_c1_full_frame(cf, layout):
    w = scenes.workload("C1")
    say(f"C1 64x64 depth, {layout}")
    from dataclasses import replace
    p = replace(w.params, jitter=1)
    sc = scenes.make_scene(w)
    vol = cf.device_volume(sc, layout=layout, occupancy=layout != "dense")
    rgba, depth = cf.cloud_render_depth(vol, w.camera(0), p, 2, 64, 64)
    plain = cf.cloud_render(vol, w.camera(0), p, 2, 64, 64)
    assert np.array_equal(to_np(rgba), to_np(plain))
    want_rgba, want_d = O.render(oracle_volume(sc), w.camera(0), p, 64, 64, frame=2,
                                 return_depth=True)
    d = to_np(depth)
    assert depth_close(d, want_d, want_rgba[..., 3]) < 1e-3
    assert np.all(d[want_d == 0.0] == 0.0)
    assert (want_d == 0.0).any() and (want_rgba[..., 3] > 0.5).any()


def test_depth_h_sampled(cf):
    w = scenes.workload("H")
    say("H 1080p depth, sampled pixels")
    sc = scenes.make_scene(w)
    vol = cf.device_volume(sc, layout="quad", occupancy=True)
    _, depth = cf.cloud_render_depth(vol, w.camera(6), w.params, 6, w.width, w.height)
    pix = scenes.random_pixels(w.width, w.height, 3000, seed=61)
    want_rgba, want_d = O.render(oracle_volume(sc), w.camera(6), w.params, w.width, w.height,
                                 frame=6, pixels=pix, return_depth=True)
    got = to_np(depth)[pix[:, 1], pix[:, 0]]
    assert depth_close(got, want_d, want_rgba[:, 3]) < 1e-3


def test_reproject_one_step_full_frame(cf):
    import torch
    w = scenes.workload("C2")
    W, H = w.width, w.height
    say(f"C2 {W}x{H}: frame 0 copy, frame 1 reprojected resolve, full frame vs oracle")
    sc = scenes.make_scene(w)
    ov = oracle_volume(sc)
    vol = cf.device_volume(sc, layout="quad", occupancy=True)
    c0, c1 = w.camera(0), w.camera(1)
    r0 = cf.cloud_render(vol, c0, w.params, 0, W, H)
    hist = torch.empty_like(r0)
    cf.cloud_taa_resolve(r0, None, hist, w.taa_blend, 0)
    r1, d1 = cf.cloud_render_depth(vol, c1, w.params, 1, W, H)
    out = cf.cloud_taa_resolve_reproject(r1, d1, hist, None, c1, c0, w.taa_blend, 1)
    o0 = O.render(ov, c0, w.params, W, H, frame=0)
    o1, od1 = O.render(ov, c1, w.params, W, H, frame=1, return_depth=True)
    want = O.taa_resolve_reproject(o1, o0, od1, c1, c0, w.taa_blend, 1)
    assert max_err(to_np(out), want) < FP32_TOL
    # the camera moved: the result differs from the plain resolve
    plain = O.taa_resolve(o1, o0, w.taa_blend, 1)
    assert np.max(np.abs(want - plain)) > 1e-2


@pytest.mark.parametrize("W,H,F", [(320, 180, 16), (640, 360, 8)])
def test_reproject_chain_orbit(cf, W, H, F):
    import torch
    w = scenes.workload("C2")
    say(f"C2 {W}x{H}: {F}-frame orbit, render_depth + reprojected resolve chain vs oracle")
    sc = scenes.make_scene(w)
    ov = oracle_volume(sc)
    vol = cf.device_volume(sc, layout="oct", occupancy=True)
    bufs = [torch.zeros((H, W, 4), device="cuda") for _ in range(2)]
    want_hist = None
    for f in range(F):
        cam, prev = w.camera(f), w.camera(max(f - 1, 0))
        cur, dep = cf.cloud_render_depth(vol, cam, w.params, f, W, H)
        cf.cloud_taa_resolve_reproject(cur, dep, bufs[(f + 1) % 2], bufs[f % 2], cam, prev,
                                       w.taa_blend, f)
        o, od = O.render(ov, cam, w.params, W, H, frame=f, return_depth=True)
        want_hist = O.taa_resolve_reproject(o, want_hist, od, cam, prev, w.taa_blend, f)
        got = to_np(bufs[f % 2])
        err = np.abs(got.astype(np.float64) - want_hist)
        say(f"  frame {f}: max-abs {err.max():.3g}, mean-abs {err.mean():.3g}")
        assert err.max() < FP32_TOL and err.mean() < 2e-6, (f, err.max(), err.mean())


def test_reproject_still_camera_matches_plain_resolve(cf):
    import torch
    w = scenes.workload("C2")
    W, H = 256, 144
    say("still camera: reprojected resolve vs the plain resolve")
    vol = cf.device_volume(scenes.make_scene(w), layout="quad")
    cam = w.camera(3)
    a = cf.cloud_render(vol, cam, w.params, 2, W, H)
    b, d = cf.cloud_render_depth(vol, cam, w.params, 3, W, H)
    plain = torch.empty_like(a)
    cf.cloud_taa_resolve(b, a, plain, w.taa_blend, 3)
    rep = cf.cloud_taa_resolve_reproject(b, d, a, None, cam, cam, w.taa_blend, 3)
    assert max_err(to_np(rep), to_np(plain)) < FP32_TOL


def test_reproject_argument_errors(cf):
    import torch
    w = scenes.workload("C2")
    say("reprojected resolve argument errors")
    vol = cf.device_volume(scenes.make_scene(w), layout="quad")
    cur, dep = cf.cloud_render_depth(vol, w.camera(1), w.params, 1, 64, 32)
    hist = torch.zeros_like(cur)
    with pytest.raises(cf.CloudError, match="in place"):
        cf.cloud_taa_resolve_reproject(cur, dep, hist, hist, w.camera(1), w.camera(0), 0.1, 1)
    with pytest.raises(cf.CloudError, match="overlaps current"):
        cf.cloud_taa_resolve_reproject(cur, dep, hist, cur, w.camera(1), w.camera(0), 0.1, 1)
    with pytest.raises(cf.CloudError, match="blend"):
        cf.cloud_taa_resolve_reproject(cur, dep, hist, None, w.camera(1), w.camera(0), 0.0, 1)
    with pytest.raises(cf.CloudError, match="depth"):
        cf.cloud_taa_resolve_reproject(cur, None, hist, None, w.camera(1), w.camera(0), 0.1, 1)
    # frame 0 copies without reading depth or cameras
    out = cf.cloud_taa_resolve_reproject(cur, None, None, None, w.camera(1), w.camera(0), 0.1, 0)
    assert np.array_equal(to_np(out), to_np(cur))

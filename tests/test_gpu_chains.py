"""Full-size temporal chains on the GPU against the oracle (Section 3.2: the
jittered frames are accumulated by the resolve), and the served FP16 form
the benchmark reports against the plain chain.

A resolved pixel depends, each frame, only on the current frame's 3x3
neighbourhood and on its own history. So the oracle follows a chain at a
sample of pixels exactly by rendering, per frame, just those pixels'
neighbourhoods (edge-clamped) and resolving each sampled pixel from its own
3x3 patch: the GPU renders every pixel at full size, the oracle a few
thousand.
"""

import sys
import time

import numpy as np
import pytest

from oracle import cloud as O
from paper_1609_05344_amd import scenes
from tests.helpers import (FP32_TOL, HALF_TOL, max_err, oracle_chain_sampled, oracle_volume,
                           to_np)

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


def gpu_chain(cf, vol, cams, params, W, H, frames, pix, blend=0.1):
    """cloud_render + cloud_taa_resolve over the frames at full size; per
    frame (current, resolved) at pix, and the last resolved frame whole."""
    import torch
    hist = torch.zeros((H, W, 4), device="cuda")
    cur = torch.empty((H, W, 4), device="cuda")
    out = []
    for k, f in enumerate(frames):
        cf.cloud_render(vol, cams[k], params, f, W, H, out=cur)
        cf.cloud_taa_resolve(cur, hist, hist, blend, 0 if k == 0 else f)
        c, h = to_np(cur), to_np(hist)
        out.append((c[pix[:, 1], pix[:, 0]].copy(), h[pix[:, 1], pix[:, 0]].copy()))
    return out, to_np(hist)


@pytest.mark.parametrize("name,layout,frames", [
    ("H", "quad", list(range(400, 416))),      # the benchmark's workload, layout and window
    ("C2", "quad", list(range(0, 16))),
    ("C2", "dense", list(range(0, 16))),
])
def test_full_size_chain_sampled(cf, name, layout, frames):
    w = scenes.workload(name)
    W, H = w.width, w.height
    say(f"chain: {name} {W}x{H} {layout} + occupancy, {len(frames)} orbit frames vs oracle")
    sc = scenes.make_scene(w)
    vol = cf.device_volume(sc, layout=layout, occupancy=True)
    cams = [w.camera(f) for f in frames]
    pix = scenes.random_pixels(W, H, 1200, seed=len(frames) + W)
    t = time.time()
    got, _ = gpu_chain(cf, vol, cams, w.params, W, H, frames, pix)
    want = oracle_chain_sampled(oracle_volume(sc), cams, w.params, W, H, frames, pix)
    say(f"  oracle chain at {len(pix)} pixels: {time.time() - t:.1f} s")
    for k in range(len(frames)):
        assert max_err(got[k][0], want[k][0]) < FP32_TOL, ("current", k)
        assert max_err(got[k][1], want[k][1]) < FP32_TOL, ("resolved", k)
    # the sample must see cloud, and the history must have moved
    assert np.mean(want[-1][1][:, 3] > 0.05) > 0.2
    assert max_err(want[-1][1], want[-1][0]) > 1e-3


def test_served_form_matches_plain_chain(cf):
    """One FP16 quad + occupancy chain at 1080p (the served benchmark's
    volume) against the oracle on its decoded volume and on the FP32 source:
    the serving tests below compare the server's frames bitwise with this
    same plain chain."""
    w = scenes.workload("H")
    W, H = w.width, w.height
    frames = [400, 401, 402, 403]
    say("chain: H FP16 quad + occupancy, 4 frames vs oracle (decoded and FP32 source)")
    sc16 = scenes.make_scene(w, dtype="f16")
    sc32 = scenes.make_scene(w, dtype="f32")
    vol = cf.device_volume(sc16, layout="quad", occupancy=True)
    cams = [w.camera(f) for f in frames]
    pix = scenes.random_pixels(W, H, 1000, seed=16)
    got, _ = gpu_chain(cf, vol, cams, w.params, W, H, frames, pix)
    dec = oracle_chain_sampled(oracle_volume(sc16), cams, w.params, W, H, frames, pix)
    src = oracle_chain_sampled(oracle_volume(sc32), cams, w.params, W, H, frames, pix)
    for k in range(len(frames)):
        assert max_err(got[k][1], dec[k][1]) < HALF_TOL, ("decoded", k)
        assert max_err(got[k][1], src[k][1]) < HALF_TOL, ("source", k)


def finish(srv, ids, timeout=120.0):
    want, got = set(ids), {}
    t0 = time.time()
    while want - set(got):
        for c in srv.poll(256):
            got[c["request_id"]] = c
        if want - set(got):
            srv.wait(0.05)
        assert time.time() - t0 < timeout, "serving timed out"
    return got


@pytest.mark.parametrize("queues,graphs,hio", [
    (1, True, False), (2, True, False), (1, False, False), (2, False, False),
    (1, True, True), (2, False, True)])
def test_served_fp16_quad_1080p_chains(cf, queues, graphs, hio):
    """The served benchmark's configuration: FP16 quad + occupancy volume, 8
    camera streams at 1920x1080, 4 chained frames each, submitted together
    so that the batches mix streams (with one queue, two frames of a stream
    in flight), the history kept by the library or read from the previous
    output (hio). Every served frame is bitwise the plain chain's
    (cloud_render + cloud_taa_resolve on the same volume), and the last
    frames of two streams match the oracle at sampled pixels."""
    import torch
    w = scenes.workload("H")
    W, H = w.width, w.height
    n_streams, frames = 8, [400, 401, 402, 403]
    say(f"serve: {n_streams} streams x {len(frames)} frames at 1080p, FP16 quad + occupancy, "
        f"queues={queues} graphs={graphs} history_in_output={hio}")
    sc = scenes.make_scene(w, dtype="f16")
    vol = cf.device_volume(sc, layout="quad", occupancy=True)

    def cam(s, f):
        return w.camera(f + 30 * s)

    outs = [[torch.zeros((H, W, 4), device="cuda") for _ in frames] for _ in range(n_streams)]
    with cf.Server(vol, budget_bytes=4 << 30, max_batch=64, queues=queues,
                   use_graphs=graphs, history_in_output=hio) as srv:
        ids = []
        for k, f in enumerate(frames):
            for s in range(n_streams):
                ids.append(srv.submit(s, cam(s, f), w.params, W, H, f, outs[s][k]))
        got = finish(srv, ids)
        assert all(c["status"] == 0 for c in got.values())
        assert srv.stats()["batches"] >= 2
    torch.cuda.synchronize()
    pix = scenes.random_pixels(W, H, 600, seed=3)
    for s in range(n_streams):
        cams = [cam(s, f) for f in frames]
        hist = torch.zeros((H, W, 4), device="cuda")
        cur = torch.empty((H, W, 4), device="cuda")
        for k, f in enumerate(frames):
            cf.cloud_render(vol, cams[k], w.params, f, W, H, out=cur)
            cf.cloud_taa_resolve(cur, hist, hist, 0.1, 0 if k == 0 else f)
            assert torch.equal(outs[s][k], hist), (s, k)
        if s in (0, 5):
            want = oracle_chain_sampled(oracle_volume(sc), cams, w.params, W, H, frames, pix)
            got_px = to_np(outs[s][-1])[pix[:, 1], pix[:, 0]]
            assert max_err(got_px, want[-1][1]) < HALF_TOL, s


@pytest.mark.parametrize("name,dtype,layout,occ", [
    ("C3", "f16", "oct", False), ("C3", "bf16", "oct", False),
    ("H", "f16", "quad", True), ("H", "bf16", "quad", True),
])
def test_half_storage_against_f32_source(cf, name, dtype, layout, occ):
    """16-bit storage's whole error -- the rounding of the stored texels plus
    the arithmetic -- against the oracle on the FP32 source volume, at sampled
    pixels of one full-size frame."""
    w = scenes.workload(name)
    W, H = w.width, w.height
    say(f"{name} {dtype} {layout} vs the oracle on the FP32 source volume")
    sc16 = scenes.make_scene(w, dtype=dtype)
    sc32 = scenes.make_scene(w, dtype="f32")
    vol = cf.device_volume(sc16, layout=layout, occupancy=occ)
    pix = scenes.random_pixels(W, H, 4000, seed=77)
    img = to_np(cf.cloud_render(vol, w.camera(400), w.params, 400, W, H))
    want = O.render(oracle_volume(sc32), w.camera(400), w.params, W, H, frame=400, pixels=pix)
    err = max_err(img[pix[:, 1], pix[:, 0]], want)
    say(f"  max-abs {err:.3g}")
    assert err < HALF_TOL


def test_served_c5_fp16_quad_4k_chains(cf):
    """The 8-view 4K served configuration: C5's FP16 512^3 quad + occupancy
    volume (above 512 MiB, so the server holds 4 render workgroups a CU), one
    stream per view, 3 frames each submitted together (two in flight), each
    stream resolving against its previous output. Every served frame is
    bitwise the plain chain's, and two streams' last frames match the oracle
    at sampled pixels."""
    import torch
    w = scenes.workload("C5")
    W, H, V = w.width, w.height, w.views
    frames = [400, 401, 402]
    say(f"serve: C5, {V} streams x {len(frames)} frames at {W}x{H}, FP16 quad + occupancy, "
        "history in the outputs")
    sc = scenes.make_scene(w, dtype="f16")
    vol = cf.device_volume(sc, layout="quad", occupancy=True)

    def cam(s, f):
        return w.camera(f, view=s)

    outs = [[torch.zeros((H, W, 4), device="cuda") for _ in frames] for _ in range(V)]
    with cf.Server(vol, budget_bytes=16 << 30, max_batch=64, history_in_output=True) as srv:
        ids = [srv.submit(s, cam(s, f), w.params, W, H, f, outs[s][k])
               for k, f in enumerate(frames) for s in range(V)]
        got = finish(srv, ids, timeout=300.0)
        assert all(c["status"] == 0 for c in got.values())
    torch.cuda.synchronize()
    pix = scenes.random_pixels(W, H, 400, seed=9)
    hist = torch.zeros((H, W, 4), device="cuda")
    cur = torch.empty((H, W, 4), device="cuda")
    for s in range(V):
        cams = [cam(s, f) for f in frames]
        for k, f in enumerate(frames):
            cf.cloud_render(vol, cams[k], w.params, f, W, H, out=cur)
            cf.cloud_taa_resolve(cur, hist, hist, 0.1, 0 if k == 0 else f)
            assert torch.equal(outs[s][k], hist), (s, k)
        if s in (0, 5):
            want = oracle_chain_sampled(oracle_volume(sc), cams, w.params, W, H, frames, pix)
            got_px = to_np(outs[s][-1])[pix[:, 1], pix[:, 0]]
            assert max_err(got_px, want[-1][1]) < HALF_TOL, s
    del outs, hist, cur
    torch.cuda.empty_cache()

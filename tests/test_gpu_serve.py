"""Serving through the C ABI on the GPU: continuous batching of many camera
streams gives, for every request, exactly the frame the plain single-frame
path (cloud_render then cloud_taa_resolve against the same history) gives --
alone or in a mix of other streams -- and that matches the oracle."""

import sys
import time
from dataclasses import replace

import numpy as np
import pytest

from oracle import cloud as O
from paper_1609_05344_amd import scenes
from tests.helpers import FP32_TOL, HALF_TOL, max_err, oracle_volume, to_np

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


@pytest.fixture(scope="module")
def vol(cf):
    w = scenes.workload("C2")
    return cf.device_volume(scenes.make_scene(w))


def finish(srv, ids, timeout=60.0):
    """Poll until every request id completed; returns {id: completion}."""
    want, got = set(ids), {}
    t0 = time.time()
    while want - set(got):
        for c in srv.poll(256):
            got[c["request_id"]] = c
        if want - set(got):
            srv.wait(0.05)
        assert time.time() - t0 < timeout, "serving timed out"
    return got


def plain_chain(cf, vol, cams, params, W, H, frames, blend=0.1):
    """Reference: cloud_render + cloud_taa_resolve per frame, one stream."""
    import torch
    hist = torch.zeros((H, W, 4), device="cuda")
    cur = torch.empty((H, W, 4), device="cuda")
    outs = []
    for k, f in enumerate(frames):
        cf.cloud_render(vol, cams[k], params, f, W, H, out=cur)
        cf.cloud_taa_resolve(cur, hist, hist, blend, 0 if k == 0 else f)
        outs.append(to_np(hist).copy())
    torch.cuda.synchronize()
    return outs


def test_one_stream_matches_plain_chain_and_oracle(cf, vol):
    import torch
    say("serve: one stream, 5 frames vs plain chain and oracle")
    w = scenes.workload("C2")
    W, H, frames = 96, 64, [3, 4, 5, 6, 7]
    cams = [w.camera(f) for f in frames]
    ref = plain_chain(cf, vol, cams, w.params, W, H, frames)
    outs = [torch.zeros((H, W, 4), device="cuda") for _ in frames]
    with cf.Server(vol, budget_bytes=1 << 30) as srv:
        # frame 3 is the stream's first request: no history, so it is copied
        ids = []
        for k, f in enumerate(frames):
            ids.append(srv.submit(1, cams[k], w.params, W, H, f, outs[k]))
        got = finish(srv, ids)
        assert all(c["status"] == 0 for c in got.values())
        for c in got.values():
            assert c["t_submit_ns"] <= c["t_admit_ns"] <= c["t_start_ns"] <= c["t_done_ns"]
        st = srv.stats()
        assert st["completed"] == 5 and st["streams"] == 1 and st["bytes_in_use"] > 0
    torch.cuda.synchronize()
    for k in range(len(frames)):
        assert np.array_equal(to_np(outs[k]), ref[k]), k
    sc = scenes.make_scene(w)
    hist = None
    for k, f in enumerate(frames):
        cur = O.render(oracle_volume(sc), cams[k], w.params, W, H, frame=f)
        hist = O.taa_resolve(cur, hist, 0.1, 0 if k == 0 else f)
    assert max_err(to_np(outs[-1]), hist) < FP32_TOL


@pytest.mark.parametrize("use_graphs", [True, False])
def test_alone_equals_mixed(cf, vol, use_graphs):
    import torch
    say(f"serve: alone vs mixed with 24 other streams (graphs={use_graphs})")
    w = scenes.workload("C2")
    rng = np.random.default_rng(7)
    W, H = 160, 90
    A_frames = [0, 1, 2]
    camsA = [scenes.orbit_camera(1.0, 200.0 + f, 10.0) for f in A_frames]
    alone = [torch.zeros((H, W, 4), device="cuda") for _ in A_frames]
    with cf.Server(vol, budget_bytes=4 << 30, use_graphs=use_graphs) as srv:
        ids = [srv.submit(42, camsA[k], w.params, W, H, f, alone[k]) for k, f in enumerate(A_frames)]
        finish(srv, ids)
    mixed = [torch.zeros((H, W, 4), device="cuda") for _ in A_frames]
    others = []
    with cf.Server(vol, budget_bytes=4 << 30, max_batch=16, use_graphs=use_graphs) as srv:
        ids = []
        for k, f in enumerate(A_frames):
            for s in range(24):
                ow, oh = [(16, 16), (37, 23), (128, 72), (320, 180)][s % 4]
                steps = [8, 16, 32][s % 3]
                p = replace(w.params, steps=steps)
                cam = scenes.orbit_camera(1.0, 100.0 + 7 * s + f, 5.0 + s % 5)
                o = torch.zeros((oh, ow, 4), device="cuda")
                others.append((s, f, cam, p, ow, oh, o))
                ids.append(srv.submit(100 + s, cam, p, ow, oh, f, o))
            ids.append(srv.submit(42, camsA[k], w.params, W, H, f, mixed[k]))
        got = finish(srv, ids)
        assert all(c["status"] == 0 for c in got.values())
        assert srv.stats()["batches"] > 1
    torch.cuda.synchronize()
    for k in range(len(A_frames)):
        assert np.array_equal(to_np(alone[k]), to_np(mixed[k])), k
    # a few of the other streams against their own plain chains
    for s in (0, 3, 5):
        seq = [x for x in others if x[0] == s]
        ref = plain_chain(cf, vol, [x[2] for x in seq], seq[0][3], seq[0][4], seq[0][5],
                          [x[1] for x in seq])
        for k, x in enumerate(seq):
            assert np.array_equal(to_np(x[6]), ref[k]), (s, k)


@pytest.mark.parametrize("same_buffer,queues", [(False, 1), (True, 1), (False, 2)])
def test_history_in_output(cf, vol, same_buffer, queues):
    """history_in_output: each stream resolves against its previous frame's
    output buffer instead of a library copy. Frames are bitwise the plain
    chain's, with one buffer per frame or one buffer reused for every frame
    (resolved in place), with the resolve on the render's queue or on its
    own; the stream state holds no history."""
    import torch
    say(f"serve: history in the outputs (same_buffer={same_buffer}, queues={queues})")
    w = scenes.workload("C2")
    W, H = 128, 72
    frames = [0, 1, 2, 3, 4, 5]
    n = 6
    cams = {s: [scenes.orbit_camera(1.0, 40.0 * s + f, 8.0) for f in frames] for s in range(n)}
    refs = {s: plain_chain(cf, vol, cams[s], w.params, W, H, frames) for s in range(n)}
    if same_buffer:
        bufs = {s: [torch.zeros((H, W, 4), device="cuda")] * len(frames) for s in range(n)}
    else:
        bufs = {s: [torch.zeros((H, W, 4), device="cuda") for _ in frames] for s in range(n)}
    with cf.Server(vol, budget_bytes=1 << 30, max_batch=8, queues=queues,
                   history_in_output=True) as srv:
        ids = [srv.submit(s, cams[s][k], w.params, W, H, f, bufs[s][k])
               for k, f in enumerate(frames) for s in range(n)]
        got = finish(srv, ids)
        assert all(c["status"] == 0 for c in got.values())
        st = srv.stats()
        # one scratch frame a stream (two with the resolve queue), no history
        assert st["bytes_in_use"] == n * queues * (((W * H * 16 + 255) // 256) * 256)
    torch.cuda.synchronize()
    for s in range(n):
        if same_buffer:
            assert np.array_equal(to_np(bufs[s][0]), refs[s][-1]), s
        else:
            for k in range(len(frames)):
                assert np.array_equal(to_np(bufs[s][k]), refs[s][k]), (s, k)


@pytest.mark.parametrize("lead_us", [-1, 0, 5000])
def test_start_lead_keeps_results(cf, vol, lead_us):
    """The batch start policy changes only when batches start: a mix of
    streams submitted as they complete gives the plain chain's frames."""
    import torch
    say(f"serve: start lead {lead_us} us, closed loop of 10 streams")
    w = scenes.workload("C2")
    W, H, n, nf = 96, 64, 10, 5
    cams = {s: [scenes.orbit_camera(1.0, 30.0 * s + f, 6.0) for f in range(nf)] for s in range(n)}
    outs = {s: [torch.zeros((H, W, 4), device="cuda") for _ in range(nf)] for s in range(n)}
    with cf.Server(vol, budget_bytes=1 << 30, start_lead_us=lead_us) as srv:
        sent = {s: 0 for s in range(n)}
        for s in range(n):
            srv.submit(s, cams[s][0], w.params, W, H, 0, outs[s][0])
        done, t0 = 0, time.time()
        while done < n * nf:
            for c in srv.poll(256):
                assert c["status"] == 0
                done += 1
                s = c["stream_id"]
                sent[s] += 1
                if sent[s] < nf:
                    k = sent[s]
                    srv.submit(s, cams[s][k], w.params, W, H, k, outs[s][k])
            srv.wait(0.01)
            assert time.time() - t0 < 60.0, "serving timed out"
    torch.cuda.synchronize()
    for s in (0, 4, 9):
        ref = plain_chain(cf, vol, cams[s], w.params, W, H, list(range(nf)))
        for k in range(nf):
            assert np.array_equal(to_np(outs[s][k]), ref[k]), (s, k)


@pytest.mark.parametrize("cap", [1, 4])
def test_render_workgroup_cap_keeps_results(cf, vol, cap):
    """serve_blocks_per_cu changes only how many persistent render workgroups
    a CU holds: the served frames stay the plain chain's."""
    import torch
    say(f"serve: {cap} render workgroups per CU, 6 streams x 3 frames")
    w = scenes.workload("C2")
    W, H, n, frames = 200, 120, 6, [0, 1, 2]
    cams = {s: [scenes.orbit_camera(1.0, 50.0 * s + f, 7.0) for f in frames] for s in range(n)}
    outs = {s: [torch.zeros((H, W, 4), device="cuda") for _ in frames] for s in range(n)}
    cf.cloud_tune("serve_blocks_per_cu", cap)
    try:
        with cf.Server(vol, budget_bytes=1 << 30) as srv:
            ids = [srv.submit(s, cams[s][k], w.params, W, H, f, outs[s][k])
                   for k, f in enumerate(frames) for s in range(n)]
            got = finish(srv, ids)
            assert all(c["status"] == 0 for c in got.values())
    finally:
        cf.cloud_tune("serve_blocks_per_cu", 0)
    torch.cuda.synchronize()
    for s in (0, 5):
        ref = plain_chain(cf, vol, cams[s], w.params, W, H, frames)
        for k in range(len(frames)):
            assert np.array_equal(to_np(outs[s][k]), ref[k]), (s, k)


def test_budget_admission_and_close(cf, vol):
    import torch
    say("serve: admission under a small budget, close_stream frees room")
    w = scenes.workload("C2")
    W, H = 64, 64
    per_stream = 2 * W * H * 16
    outs = {s: torch.zeros((H, W, 4), device="cuda") for s in range(4)}
    with cf.Server(vol, budget_bytes=2 * per_stream) as srv:
        rc, _ = srv.try_submit(9, w.camera(0), w.params, 256, 256, 0,
                               torch.zeros((256, 256, 4), device="cuda"))
        assert rc == -2                       # can never fit
        ids = {s: srv.submit(s, w.camera(s), w.params, W, H, 1, outs[s]) for s in range(4)}
        got = {}
        t0 = time.time()
        while len(got) < 2 and time.time() - t0 < 10:
            for c in srv.poll():
                got[c["request_id"]] = c
            srv.wait(0.05)
        time.sleep(0.1)
        for c in srv.poll():
            got[c["request_id"]] = c
        assert len(got) == 2                  # only two streams fit
        st = srv.stats()
        assert st["bytes_in_use"] == 2 * per_stream and st["queued"] == 2
        done_streams = {c["stream_id"] for c in got.values()}
        for s in done_streams:
            assert srv.close_stream(s) == 0
        rest = finish(srv, [ids[s] for s in range(4) if s not in done_streams])
        assert all(c["status"] == 0 for c in rest.values())
        assert srv.close_stream(12345) == -5
    torch.cuda.synchronize()


def test_argument_errors(cf, vol):
    import torch
    w = scenes.workload("C2")
    out = torch.zeros((32, 32, 4), device="cuda")
    with cf.Server(vol, budget_bytes=1 << 30) as srv:
        rc, _ = srv.try_submit(1, w.camera(0), w.params, 32, 32, 0, None)
        assert rc == -1
        rc, _ = srv.try_submit(1, w.camera(0), replace(w.params, steps=0), 32, 32, 0, out)
        assert rc == -1
        rid = srv.submit(1, w.camera(0), w.params, 32, 32, 0, out)
        rc, _ = srv.try_submit(1, w.camera(1), w.params, 16, 16, 1, out)
        assert rc == -1                       # resolution fixed by the first request
        finish(srv, [rid])
    with pytest.raises(cf.CloudError):
        cf.Server(vol, budget_bytes=1 << 30, max_batch=65)


def test_fp16_oct_server_1080p(cf):
    import torch
    w = scenes.workload("H")
    say("serve: f16 oct volume, 4 streams at 1080p vs oracle (sampled)")
    sc = scenes.make_scene(w, dtype="f16")
    packed = cf.cloud_volume_pack(cf.device_volume(sc), "oct")
    outs = [torch.zeros((w.height, w.width, 4), device="cuda") for _ in range(4)]
    with cf.Server(packed, budget_bytes=8 << 30) as srv:
        ids = [srv.submit(s, w.camera(10 * s), w.params, w.width, w.height, 0, outs[s])
               for s in range(4)]
        got = finish(srv, ids)
        assert all(c["status"] == 0 for c in got.values())
    torch.cuda.synchronize()
    pix = scenes.random_pixels(w.width, w.height, 1500, seed=5)
    for s in (0, 3):
        want = O.render(oracle_volume(sc), w.camera(10 * s), w.params, w.width, w.height,
                        frame=0, pixels=pix)
        got = to_np(outs[s])[pix[:, 1], pix[:, 0]]
        assert max_err(got, want) < HALF_TOL


def test_poll_with_a_huge_max_returns_a_code(cf, vol):
    """cloud_serve_poll allocates nothing that grows with max: an idle
    server, and one with two finished requests, polled with the largest max
    into a small array, return CLOUD_OK with the right counts."""
    import ctypes
    import torch
    from paper_1609_05344_amd import _lib
    say("serve: poll with max = 2^31 - 1")
    w = scenes.workload("C2")
    outs = [torch.zeros((32, 32, 4), device="cuda") for _ in range(2)]
    arr = (_lib.cloud_completion * 8)()
    n = ctypes.c_int32(-1)
    with cf.Server(vol, budget_bytes=1 << 30) as srv:
        rc = srv.lib.cloud_serve_poll(srv.handle, arr, 2**31 - 1, ctypes.byref(n))
        assert rc == 0 and n.value == 0
        ids = [srv.submit(s, w.camera(s), w.params, 32, 32, 0, outs[s]) for s in range(2)]
        while srv.stats()["completed"] < 2:
            srv.wait(0.05)
        rc = srv.lib.cloud_serve_poll(srv.handle, arr, 2**31 - 1, ctypes.byref(n))
        assert rc == 0 and n.value == 2
        assert sorted(arr[i].request_id for i in range(2)) == sorted(ids)
        assert all(arr[i].status == 0 for i in range(2))

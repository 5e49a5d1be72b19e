"""Lookup trace, gather record and gather replay, through the C ABI.

The trace records which lookups the render performs. It must add up to the
render's own lookup count and agree per pixel with the oracle's trace, up to
the few samples whose density or early exit lands on the other side of zero
or t_eps in float32 than in float64. The record holds those lookups as texel
corners per wavefront slot; the replay is a measurement kernel that fetches
them: it must be deterministic, independent of residency, fetch nothing for
lanes without lookups, run for every dtype and layout, and reject what it
does not support. Its output has no meaning beyond keeping every fetch alive.
"""

import sys
from dataclasses import replace

import numpy as np
import pytest

from oracle import cloud as O
from paper_1609_05344_amd import scenes
from tests.helpers import oracle_volume, to_np

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


def split(trace):
    a = to_np(trace).view(np.uint32)
    return a[..., 0], a[..., 1]


def popcount(m):
    m = m.astype(np.uint64)
    return sum(((m >> np.uint64(k)) & np.uint64(1)) for k in range(32)).astype(np.int64)


@pytest.mark.parametrize("layout,occ", [("dense", False), ("quad", True), ("oct", True)])
def test_trace_adds_up_to_count(cf, layout, occ):
    w = scenes.workload("H")
    say(f"trace vs count, H 320x180, {layout} occupancy={occ}")
    sc = scenes.make_scene(w)
    vol = cf.device_volume(sc, layout=layout, occupancy=occ)
    prim, mask = split(cf.cloud_lookup_trace(vol, [w.camera(1)], w.params, 1, 320, 180))
    count = int(to_np(cf.cloud_count_lookups(vol, w.camera(1), w.params, 1, 320, 180))[0])
    assert prim.shape == (1, 180, 320)
    assert int(prim.sum()) + w.params.light_steps * int(popcount(mask).sum()) == count
    assert prim.max() <= w.params.steps
    assert np.all((mask.astype(np.uint64) >> prim.astype(np.uint64)) == 0)
    assert 0.3 < (prim > 0).mean() < 1.0


def test_trace_matches_oracle(cf):
    w = scenes.workload("H")
    W, H = 160, 90
    say(f"trace vs oracle trace, H {W}x{H} frame 2")
    sc = scenes.make_scene(w)
    prim, mask = split(cf.cloud_lookup_trace(cf.device_volume(sc), [w.camera(2)], w.params, 2, W, H))
    _, (oprim, omask) = O.render(oracle_volume(sc), w.camera(2), w.params, W, H, frame=2,
                                 return_trace=True)
    differ = (prim[0].reshape(-1) != oprim) | (mask[0].reshape(-1).astype(np.uint64) != omask)
    assert differ.mean() <= 2e-3, differ.sum()
    assert (oprim > 0).mean() > 0.3


def test_trace_views_equal_single_view_traces(cf):
    w = scenes.workload("C2")
    say("trace of 3 views in one launch vs one view at a time")
    sc = scenes.make_scene(w, dtype="f16")
    vol = cf.device_volume(sc, layout="oct", occupancy=True)
    cams = [w.camera(4, view=v) for v in range(3)]
    multi = to_np(cf.cloud_lookup_trace(vol, cams, w.params, 4, 200, 120))
    for v in range(3):
        one = to_np(cf.cloud_lookup_trace(vol, [cams[v]], w.params, 4, 200, 120))
        assert np.array_equal(multi[v], one[0])


def _valid_codes(codes, counts):
    """The recorded codes of each wavefront's used slots, as uint32 [n, 64]."""
    c = to_np(codes).view(np.uint32)
    n = to_np(counts).view(np.uint32)
    used = np.arange(c.shape[1])[None, :] < n[:, None]
    return c[used], n


@pytest.mark.parametrize("layout", ["dense", "quad", "oct"])
def test_record_matches_the_render(cf, layout):
    """The recorded slots hold exactly the render's lookups: one code per
    executed lookup, every used slot has a lane in it, no wavefront exceeds
    steps * (1 + L) slots, corners lie in the volume, and a corner marked dead
    lies in an empty brick of the occupancy bitmap."""
    w = scenes.workload("H")
    W, H = 320, 180
    say(f"gather record vs lookup count, H {W}x{H}, {layout}")
    sc = scenes.make_scene(w)
    vol = cf.device_volume(sc, layout=layout, occupancy=True)
    cams = [w.camera(5)]
    tr = cf.cloud_lookup_trace(vol, cams, w.params, 5, W, H)
    codes, counts = cf.cloud_gather_record(vol, cams, w.params, 5, W, H, tr)
    valid, n = _valid_codes(codes, counts)
    count = int(to_np(cf.cloud_count_lookups(vol, cams[0], w.params, 5, W, H))[0])
    take = valid != 0xFFFFFFFF
    assert int(take.sum()) == count
    assert np.all(take.any(axis=1))
    assert n.max() <= w.params.steps * (1 + w.params.light_steps)
    assert n.shape[0] == cf.gather_waves(1, W, H)
    c = valid[take]
    kx, ky, kz = c & 1023, (c >> 10) & 1023, (c >> 20) & 1023
    nz, ny, nx = sc.base_f64.shape
    assert kx.max() < nx and ky.max() < ny and kz.max() < nz
    dead = ((c >> 30) & 1).astype(bool)
    assert 0.05 < dead.mean() < 0.95
    # a dead corner's brick holds no non-zero texel in [k, k + 2^lg] per axis
    lg = vol.struct.occupancy_log2
    rho = sc.base_f64
    for x, y, z in list(zip(kx[dead], ky[dead], kz[dead]))[:: max(1, int(dead.sum()) // 300)]:
        bx, by, bz = (int(x) >> lg) << lg, (int(y) >> lg) << lg, (int(z) >> lg) << lg
        e = 1 << lg
        assert not rho[bz:bz + e + 1, by:by + e + 1, bx:bx + e + 1].any()


def test_record_views_equal_single_view_records(cf):
    w = scenes.workload("C2")
    say("gather record of 3 views in one launch vs one view at a time")
    sc = scenes.make_scene(w, dtype="f16")
    vol = cf.device_volume(sc, layout="quad", occupancy=True)
    cams = [w.camera(4, view=v) for v in range(3)]
    W, H = 200, 120
    tr = cf.cloud_lookup_trace(vol, cams, w.params, 4, W, H)
    codes, counts = cf.cloud_gather_record(vol, cams, w.params, 4, W, H, tr)
    per = cf.gather_waves(1, W, H)
    for v in range(3):
        t1 = cf.cloud_lookup_trace(vol, [cams[v]], w.params, 4, W, H)
        c1, n1 = cf.cloud_gather_record(vol, [cams[v]], w.params, 4, W, H, t1)
        a, na = _valid_codes(codes[v * per:(v + 1) * per], counts[v * per:(v + 1) * per])
        b, nb = _valid_codes(c1, n1)
        assert np.array_equal(na, nb) and np.array_equal(a, b)


@pytest.mark.parametrize("dtype,layout", [("f32", "dense"), ("f32", "quad"), ("f32", "oct"),
                                          ("f16", "quad"), ("f16", "oct"), ("bf16", "quad")])
def test_replay_deterministic_any_residency(cf, dtype, layout):
    """The replay's output (an XOR of every word fetched per lane) does not
    depend on residency, repeats exactly, is zero for lanes with no lookups,
    and the random mode fetches elsewhere."""
    w = scenes.workload("H")
    say(f"gather replay H 1080p, {dtype} {layout}")
    sc = scenes.make_scene(w, dtype=dtype)
    vol = cf.device_volume(sc, layout=layout, occupancy=layout != "dense")
    cams = [w.camera(3)]
    W, H = w.width, w.height
    tr = cf.cloud_lookup_trace(vol, cams, w.params, 3, W, H)
    codes, counts = cf.cloud_gather_record(vol, cams, w.params, 3, W, H, tr)
    valid = to_np(counts).view(np.uint32)
    a = to_np(cf.cloud_gather_replay(vol, 1, W, H, codes, counts, mode=0)).view(np.uint32)
    b = to_np(cf.cloud_gather_replay(vol, 1, W, H, codes, counts, mode=0,
                                     blocks_per_cu=2)).view(np.uint32)
    r = to_np(cf.cloud_gather_replay(vol, 1, W, H, codes, counts, mode=1)).view(np.uint32)
    assert np.array_equal(a, b)
    assert np.all(a[valid == 0] == 0) and np.all(r[valid == 0] == 0)
    assert np.any(a != 0) and np.any(a != r)


def test_replay_rejects_unsupported(cf):
    import torch
    say("gather record and replay argument errors")
    w = scenes.workload("H")
    sc = scenes.make_scene(w)
    vol = cf.device_volume(sc, layout="quad")
    tr = cf.cloud_lookup_trace(vol, [w.camera(0)], w.params, 0, 64, 32)
    codes, counts = cf.cloud_gather_record(vol, [w.camera(0)], w.params, 0, 64, 32, tr)
    with pytest.raises(cf.CloudError, match="mode"):
        cf.cloud_gather_replay(vol, 1, 64, 32, codes, counts, mode=2)
    with pytest.raises(cf.CloudError, match="blocks_per_cu"):
        cf.cloud_gather_replay(vol, 1, 64, 32, codes, counts, blocks_per_cu=65)
    with pytest.raises(cf.CloudError, match="max_slots"):
        cf.cloud_gather_record(vol, [w.camera(0)], w.params, 0, 64, 32, tr, max_slots=55)
    long = replace(w.params, steps=33)
    with pytest.raises(cf.CloudError, match="steps <= 32"):
        cf.cloud_lookup_trace(vol, [w.camera(0)], long, 0, 64, 32)
    with pytest.raises(cf.CloudError, match="steps <= 32"):
        cf.cloud_gather_record(vol, [w.camera(0)], long, 0, 64, 32, tr, max_slots=33 * 7)
    shifted = torch.zeros(64 * 32 * 2 + 1, dtype=torch.int32, device="cuda")[1:]
    with pytest.raises(cf.CloudError, match="aligned"):
        cf.cloud_gather_record(vol, [w.camera(0)], w.params, 0, 64, 32, shifted)
    small = torch.zeros((cf.gather_waves(1, 64, 32), 8, 64), dtype=torch.int32, device="cuda")
    with pytest.raises(cf.CloudError, match="max_slots"):
        cf.cloud_gather_record(vol, [w.camera(0)], w.params, 0, 64, 32, tr, max_slots=8,
                               codes=small)
    c3 = scenes.workload("C3")
    dvol = cf.device_volume(scenes.make_scene(c3, dtype="f16"))
    with pytest.raises(cf.CloudError, match="detail"):
        cf.cloud_gather_replay(dvol, 1, 64, 32, codes, counts)

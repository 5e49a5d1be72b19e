"""Lookup trace and gather ceiling, through the C ABI.

The trace records which lookups the render performs. It must add up to the
render's own lookup count and agree per pixel with the oracle's trace, up to
the few samples whose density or early exit lands on the other side of zero
or t_eps in float32 than in float64. The gather ceiling is a measurement
kernel: it must be deterministic, fetch nothing for pixels without lookups,
run for every dtype and layout, and reject what it does not support. Its
output has no meaning beyond keeping every fetch alive.
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


@pytest.mark.parametrize("dtype,layout", [("f32", "dense"), ("f32", "quad"), ("f32", "oct"),
                                          ("f16", "oct"), ("bf16", "quad")])
def test_ceiling_deterministic_and_empty_pixels(cf, dtype, layout):
    w = scenes.workload("H")
    say(f"gather ceiling H 1080p, {dtype} {layout}")
    sc = scenes.make_scene(w, dtype=dtype)
    vol = cf.device_volume(sc, layout=layout, occupancy=layout != "dense")
    cams = [w.camera(3)]
    tr = cf.cloud_lookup_trace(vol, cams, w.params, 3, w.width, w.height)
    prim, _ = split(tr)
    for mode in (0, 1):
        a = to_np(cf.cloud_gather_ceiling(vol, cams, w.params, 3, w.width, w.height, tr, mode))
        b = to_np(cf.cloud_gather_ceiling(vol, cams, w.params, 3, w.width, w.height, tr, mode))
        bits = a[..., 0].view(np.uint32)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
        assert np.all(a[..., 1:] == 0)
        assert np.all(bits[prim == 0] == 0)
        assert np.any(bits[prim > 0] != 0)


def test_ceiling_rejects_unsupported(cf):
    import torch
    say("gather ceiling argument errors")
    w = scenes.workload("H")
    sc = scenes.make_scene(w)
    vol = cf.device_volume(sc, layout="quad")
    tr = cf.cloud_lookup_trace(vol, [w.camera(0)], w.params, 0, 64, 32)
    with pytest.raises(cf.CloudError, match="mode"):
        cf.cloud_gather_ceiling(vol, [w.camera(0)], w.params, 0, 64, 32, tr, 2)
    long = replace(w.params, steps=33)
    with pytest.raises(cf.CloudError, match="steps <= 32"):
        cf.cloud_lookup_trace(vol, [w.camera(0)], long, 0, 64, 32)
    with pytest.raises(cf.CloudError, match="steps <= 32"):
        cf.cloud_gather_ceiling(vol, [w.camera(0)], long, 0, 64, 32, tr, 0)
    shifted = torch.zeros(64 * 32 * 2 + 1, dtype=torch.int32, device="cuda")[1:]
    with pytest.raises(cf.CloudError, match="aligned"):
        cf.cloud_gather_ceiling(vol, [w.camera(0)], w.params, 0, 64, 32, shifted, 0)
    c3 = scenes.workload("C3")
    dvol = cf.device_volume(scenes.make_scene(c3, dtype="f16"))
    with pytest.raises(cf.CloudError, match="detail"):
        cf.cloud_gather_ceiling(dvol, [c3.camera(0)], c3.params, 0, 64, 32, tr, 0)

"""Packed volume layouts and lookup counting, through the C ABI.

The quad and oct layouts hold the same texel values as the dense volume, so
a render from a packed volume must equal the dense render bit for bit (and
therefore match the oracle to the same tolerance). The lookup count must
equal the oracle's count of the lookups it performs, up to the few samples
whose density or early exit lands on the other side of zero or t_eps in
float32 than in float64.
"""

import sys
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


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("layout", ["quad", "oct"])
def test_packed_equals_dense(cf, dtype, layout):
    w = scenes.workload("H")
    say(f"{layout} {dtype}: H frame vs dense, bitwise")
    sc = scenes.make_scene(w, dtype=dtype)
    dense = cf.device_volume(sc)
    packed = cf.cloud_volume_pack(dense, layout)
    a = to_np(cf.cloud_render(dense, w.camera(5), w.params, 5, w.width, w.height))
    b = to_np(cf.cloud_render(packed, w.camera(5), w.params, 5, w.width, w.height))
    assert np.array_equal(a, b)
    assert a[..., 3].max() > 0.5


@pytest.mark.parametrize("brick", [(3, 0, 0), (0, 3, 0), (0, 0, 3), (1, 0, 2), (2, 1, 0)])
@pytest.mark.parametrize("layout", ["quad", "oct"])
def test_brick_shapes_render_bitwise_equal(cf, layout, brick):
    w = scenes.workload("H")
    say(f"{layout} bricks {brick}: 640x360 frames vs dense, bitwise; a 32^3 volume (odd entry counts) too")
    for sc in (scenes.make_scene(w, dtype="f16"), scenes.make_scene(scenes.workload("C1"))):
        dense = cf.device_volume(sc)
        packed = cf.cloud_volume_pack(dense, layout, brick=brick)
        assert list(packed.struct.brick_log2) == list(brick)
        cam = w.camera(5) if sc.workload.name == "H" else sc.workload.camera(0)
        a = to_np(cf.cloud_render(dense, cam, w.params, 5, 640, 360))
        b = to_np(cf.cloud_render(packed, cam, w.params, 5, 640, 360))
        assert np.array_equal(a, b)
        assert a[..., 3].max() > 0.3


@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("layout", ["quad", "oct"])
def test_packed_small_volumes_vs_oracle(cf, dtype, layout):
    say(f"{layout} {dtype}: C1 full frame and odd-sized volume vs oracle")
    w = scenes.workload("C1", jitter=1)
    tol = FP32_TOL if dtype == "f32" else HALF_TOL
    sc = scenes.make_scene(w, dtype=dtype)
    packed = cf.cloud_volume_pack(cf.device_volume(sc), layout)
    got = to_np(cf.cloud_render(packed, w.camera(0), w.params, 2, 64, 64))
    assert max_err(got, O.render(oracle_volume(sc), w.camera(0), w.params, 64, 64, frame=2)) < tol
    # non-cubic, odd dims: exercises every clamped edge entry
    rng = np.random.default_rng(3)
    base = np.clip(rng.uniform(-0.5, 1.0, size=(5, 7, 3)), 0, 1)
    st = scenes.quantise(base, dtype)
    sc2 = scenes.Scene(w, st, scenes.decode(st, dtype))
    packed2 = cf.cloud_volume_pack(cf.device_volume(sc2), layout)
    cam = scenes.orbit_camera(1.2, 200.0, 35.0)
    got = to_np(cf.cloud_render(packed2, cam, w.params, 1, 40, 30))
    assert max_err(got, O.render(oracle_volume(sc2), cam, w.params, 40, 30, frame=1)) < tol


def test_pack_errors(cf):
    import torch
    w = scenes.workload("C1")
    dense = cf.device_volume(scenes.make_scene(w))
    with pytest.raises(cf.CloudError):
        cf.cloud_volume_pack(dense, "dense")
    # 2x2x2-entry bricks: each entry axis rounded up to an even count
    n = cf.cloud_volume_packed_bytes(dense, "oct")
    assert n == 34 * 34 * 34 * 8 * 4
    assert cf.cloud_volume_packed_bytes(dense, "quad") == 34 * 34 * 32 * 4 * 4
    small = torch.empty((n // 2,), dtype=torch.uint8, device="cuda")
    from paper_1609_05344_amd import _lib
    import ctypes
    out = _lib.cloud_volume()
    rc = _lib.load().cloud_volume_pack(ctypes.byref(dense.struct), 2, small.data_ptr(), n // 2,
                                       ctypes.byref(out), None)
    assert rc == _lib.CLOUD_E_INVALID and "smaller" in _lib.last_error()


@pytest.mark.parametrize("name,npix", [("C1", None), ("H", None)])
def test_lookup_count_matches_oracle(cf, name, npix):
    w = scenes.workload(name)
    say(f"lookup count {name}")
    sc = scenes.make_scene(w)
    W, H = (w.width, w.height) if name == "C1" else (320, 180)
    got = int(to_np(cf.cloud_count_lookups(cf.device_volume(sc), w.camera(1), w.params, 1, W, H))[0])
    _, want = O.render(oracle_volume(sc), w.camera(1), w.params, W, H, frame=1, return_lookups=True)
    assert want > 0
    assert abs(got - want) <= 2e-3 * want, (got, want)
    packed = cf.cloud_volume_pack(cf.device_volume(sc), "oct")
    got2 = int(to_np(cf.cloud_count_lookups(packed, w.camera(1), w.params, 1, W, H))[0])
    assert got2 == got


# ---------------------------------------------------------------------------
# occupancy bitmap: exact empty-space skipping
# ---------------------------------------------------------------------------

def occupancy_reference(base_f64, lg):
    """Brick occupancy from the definition: a brick is occupied when any texel
    of [k, k + 2^lg] (clamped) per axis, k its first texel, is non-zero."""
    nz, ny, nx = base_f64.shape
    B = 1 << lg
    nb = [((n - 1) >> lg) + 1 for n in (nx, ny, nz)]
    bits = np.zeros(nb[0] * nb[1] * nb[2], dtype=bool)
    for bz in range(nb[2]):
        for by in range(nb[1]):
            for bx in range(nb[0]):
                blk = base_f64[bz * B:min(bz * B + B, nz - 1) + 1, by * B:min(by * B + B, ny - 1) + 1,
                               bx * B:min(bx * B + B, nx - 1) + 1]
                bits[(bz * nb[1] + by) * nb[0] + bx] = bool(np.any(blk != 0))
    return bits


@pytest.mark.parametrize("name,dtype", [("C1", "f32"), ("C3", "f16")])
def test_occupancy_bitmap_matches_definition(cf, name, dtype):
    say(f"occupancy bitmap {name} {dtype}")
    w = scenes.workload(name)
    sc = scenes.make_scene(w, dtype=dtype)
    vol = cf.cloud_volume_occupancy(cf.device_volume(sc))
    lg = vol.struct.occupancy_log2
    words = to_np(vol.occupancy).view(np.uint32)
    got = ((words[:, None] >> np.arange(32)[None, :]) & 1).reshape(-1).astype(bool)
    want = occupancy_reference(sc.base_f64, lg)
    assert np.array_equal(got[:want.size], want)
    assert not got[want.size:].any()
    assert 0 < want.mean() < 1


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("layout", ["dense", "quad", "oct"])
def test_occupancy_skipping_is_exact(cf, dtype, layout):
    w = scenes.workload("H")
    say(f"occupancy skip {layout} {dtype}: H frame bitwise vs no skipping")
    sc = scenes.make_scene(w, dtype=dtype)
    plain = cf.device_volume(sc, layout=layout)
    skip = cf.device_volume(sc, layout=layout, occupancy=True)
    assert skip.struct.occupancy
    a = to_np(cf.cloud_render(plain, w.camera(7), w.params, 7, w.width, w.height))
    b = to_np(cf.cloud_render(skip, w.camera(7), w.params, 7, w.width, w.height))
    assert np.array_equal(a, b)
    na = int(to_np(cf.cloud_count_lookups(plain, w.camera(7), w.params, 7, 320, 180))[0])
    nb = int(to_np(cf.cloud_count_lookups(skip, w.camera(7), w.params, 7, 320, 180))[0])
    assert na == nb          # the method's lookups are the same; only fetches are skipped


def test_occupancy_with_detail_and_odd_volume(cf):
    say("occupancy skip: C3 with detail, and an odd-sized sparse volume vs oracle")
    w = scenes.workload("C3")
    sc = scenes.make_scene(w)
    plain, skip = cf.device_volume(sc), cf.device_volume(sc, layout="oct", occupancy=True)
    a = to_np(cf.cloud_render(plain, w.camera(0), w.params, 0, 480, 270))
    b = to_np(cf.cloud_render(skip, w.camera(0), w.params, 0, 480, 270))
    assert np.array_equal(a, b)
    rng = np.random.default_rng(11)
    base = np.where(rng.uniform(size=(21, 13, 35)) > 0.93, rng.uniform(size=(21, 13, 35)), 0.0)
    st = scenes.quantise(base, "f32")
    sc2 = scenes.Scene(scenes.workload("C1"), st, scenes.decode(st, "f32"))
    cam = scenes.orbit_camera(1.3, 230.0, 25.0)
    p = scenes.workload("C1", jitter=1).params
    for layout in ("dense", "quad", "oct"):
        v = cf.device_volume(sc2, layout=layout, occupancy=True)
        got = to_np(cf.cloud_render(v, cam, p, 3, 48, 40))
        assert max_err(got, O.render(oracle_volume(sc2), cam, p, 48, 40, frame=3)) < FP32_TOL


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_packed_detail_matches_dense_and_oracle(cf, dtype):
    say(f"packed detail {dtype}: non-power-of-two detail dims, quad and oct, vs dense and oracle")
    rng = np.random.default_rng(21)
    base = np.clip(rng.uniform(-0.2, 1.0, size=(18, 12, 20)), 0, 1)
    det = rng.uniform(0, 1, size=(6, 5, 7))
    w = scenes.workload("C3")
    bs, ds = scenes.quantise(base, dtype), scenes.quantise(det, dtype)
    sc = scenes.Scene(w, bs, scenes.decode(bs, dtype), ds, scenes.decode(ds, dtype))
    cam = scenes.orbit_camera(1.4, 215.0, 18.0)
    dense = to_np(cf.cloud_render(cf.device_volume(sc), cam, w.params, 2, 64, 48))
    for layout in ("quad", "oct"):
        v = cf.device_volume(sc, layout=layout, occupancy=True)
        assert np.array_equal(to_np(cf.cloud_render(v, cam, w.params, 2, 64, 48)), dense)
    tol = FP32_TOL if dtype == "f32" else HALF_TOL
    assert max_err(dense, O.render(oracle_volume(sc), cam, w.params, 64, 48, frame=2)) < tol


@pytest.mark.parametrize("dims", [(1024, 3, 1023), (1025, 3, 2), (2, 1030, 3), (3, 2, 1024)])
def test_index_tables_and_their_limits(cf, dims):
    # packed volumes of at most 1024 texels along x and y and fewer along z are
    # indexed through entry-index tables in LDS, larger ones by the index
    # arithmetic: both sides of each limit, packed against dense bitwise and
    # against the oracle
    nx, ny, nz = dims
    say(f"volume {dims}: quad and oct vs dense, and vs the oracle")
    w = scenes.workload("C1", jitter=1)
    rng = np.random.default_rng(nx + 7 * ny + 13 * nz)
    base = np.clip(rng.uniform(-0.3, 1.0, size=(nz, ny, nx)), 0, 1)
    st = scenes.quantise(base, "f32")
    sc = scenes.Scene(w, st, scenes.decode(st, "f32"))
    cam = scenes.orbit_camera(1.6, 205.0, 30.0)
    dense = to_np(cf.cloud_render(cf.device_volume(sc), cam, w.params, 2, 48, 40))
    for layout in ("quad", "oct"):
        got = to_np(cf.cloud_render(cf.device_volume(sc, layout=layout, occupancy=True), cam, w.params,
                                    2, 48, 40))
        assert np.array_equal(got, dense), layout
    want = O.render(oracle_volume(sc), cam, w.params, 48, 40, frame=2)
    assert max_err(dense, want) < FP32_TOL
    assert want[..., 3].max() > 0.05

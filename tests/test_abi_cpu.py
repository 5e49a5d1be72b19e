"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/*.h, its structs have the layout the binding assumes, and
argument errors that precede any device call are reported as documented."""

import ctypes
import glob
import os
import re
import subprocess

import pytest

from paper_1609_05344_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1609_05344_amd.build import build
        build()
    return _lib.load()


def declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^[A-Za-z_][\w \t\*]*?\b(cloud_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_exports_every_declared_function(lib):
    names = declared_functions()
    assert len(names) >= 6
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert lib.cloud_abi_version() == _lib.ABI_VERSION == 5


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "sizes.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "cloud.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(cloud_volume),"
        " sizeof(cloud_camera), sizeof(cloud_params), offsetof(cloud_volume, layout),"
        " offsetof(cloud_params, t_eps), offsetof(cloud_volume, detail),"
        " sizeof(cloud_serve_config), offsetof(cloud_serve_config, queues),"
        " offsetof(cloud_serve_config, start_lead_us));return 0;}\n")
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert got == [ctypes.sizeof(_lib.cloud_volume), ctypes.sizeof(_lib.cloud_camera),
                   ctypes.sizeof(_lib.cloud_params), _lib.cloud_volume.layout.offset,
                   _lib.cloud_params.t_eps.offset, _lib.cloud_volume.detail.offset,
                   ctypes.sizeof(_lib.cloud_serve_config), _lib.cloud_serve_config.queues.offset,
                   _lib.cloud_serve_config.start_lead_us.offset]


def test_argument_errors_before_any_launch(lib):
    cam = _lib.cloud_camera()
    prm = _lib.cloud_params()
    rc = lib.cloud_render(None, ctypes.byref(cam), ctypes.byref(prm), 0, 8, 8, None, None)
    assert rc == _lib.CLOUD_E_INVALID and "volume is NULL" in _lib.last_error()
    vol = _lib.cloud_volume()
    rc = lib.cloud_render(ctypes.byref(vol), None, ctypes.byref(prm), 0, 8, 8, None, None)
    assert rc == _lib.CLOUD_E_INVALID and "camera" in _lib.last_error()
    rc = lib.cloud_render(ctypes.byref(vol), ctypes.byref(cam), ctypes.byref(prm), 0, 0, 8, None, None)
    assert rc == _lib.CLOUD_E_INVALID and "width" in _lib.last_error()
    vol.dtype = 7
    rc = lib.cloud_render(ctypes.byref(vol), ctypes.byref(cam), ctypes.byref(prm), 0, 8, 8, None, None)
    assert rc == _lib.CLOUD_E_INVALID and "dtype" in _lib.last_error()
    vol.dtype, vol.layout = 0, 3
    rc = lib.cloud_render(ctypes.byref(vol), ctypes.byref(cam), ctypes.byref(prm), 0, 8, 8, None, None)
    assert rc == _lib.CLOUD_E_INVALID and "layout" in _lib.last_error()
    rc = lib.cloud_taa_resolve(None, None, None, 8, 8, 1.5, 1, None)
    assert rc == _lib.CLOUD_E_INVALID and "blend" in _lib.last_error()
    rc = lib.cloud_taa_resolve(None, None, None, 8, -1, 0.1, 1, None)
    assert rc == _lib.CLOUD_E_INVALID
    rc = lib.cloud_march_rays(ctypes.byref(vol), None, None, None, -1, ctypes.byref(prm), 0, None, None)
    assert rc == _lib.CLOUD_E_INVALID
    rc = lib.cloud_render_views(ctypes.byref(vol), ctypes.byref(cam), 0, ctypes.byref(prm), 0, 8, 8,
                                None, None)
    assert rc == _lib.CLOUD_E_INVALID and "n_views" in _lib.last_error()
    rc = lib.cloud_render_resolve(ctypes.byref(vol), None, 1, ctypes.byref(prm), 1, 8, 8, None,
                                  None, None, None, ctypes.c_float(0.1), 0, None)
    assert rc == _lib.CLOUD_E_INVALID and "cameras" in _lib.last_error()
    rc = lib.cloud_render_resolve(ctypes.byref(vol), ctypes.byref(cam), 0, ctypes.byref(prm), 1, 8,
                                  8, None, None, None, None, ctypes.c_float(0.1), 0, None)
    assert rc == _lib.CLOUD_E_INVALID and "n_views" in _lib.last_error()
    rc = lib.cloud_render_resolve(ctypes.byref(vol), ctypes.byref(cam), 1, ctypes.byref(prm), 1, 8,
                                  0, None, None, None, None, ctypes.c_float(0.1), 0, None)
    assert rc == _lib.CLOUD_E_INVALID and "height" in _lib.last_error()
    # a successful-looking call leaves the error text of the last failure only
    assert lib.cloud_jitter_offsets(None, 0, 0, 0, None, None) == _lib.CLOUD_OK


def test_packed_bytes_and_brick_shapes(lib):
    # a host-side size query: no device memory is touched
    vol = _lib.cloud_volume()
    vol.nx, vol.ny, vol.nz, vol.dtype = 32, 20, 9, 1       # f16
    n = ctypes.c_uint64(0)

    def size(layout, brick):
        vol.brick_log2[:] = list(brick)
        rc = lib.cloud_volume_packed_bytes(ctypes.byref(vol), layout, ctypes.byref(n))
        return rc, int(n.value)

    def up(e, b):
        return -(-e // (1 << b)) << b

    ex, ey = 33, 21
    for brick in ((1, 1, 1), (2, 0, 1), (3, 0, 0), (0, 0, 3), (1, 0, 2)):
        for layout, ez, corners in ((1, 9, 4), (2, 10, 8)):
            rc, got = size(layout, brick)
            assert rc == _lib.CLOUD_OK
            want = up(ex, brick[0]) * up(ey, brick[1]) * up(ez, brick[2]) * corners * 2
            assert got == want, (brick, layout, got, want)
    assert size(1, (0, 0, 0)) == size(1, (1, 1, 1))      # all zero = the default shape
    for bad in ((1, 1, 0), (2, 2, 0), (4, 0, -1), (-1, 2, 2)):
        rc, _ = size(2, bad)
        assert rc == _lib.CLOUD_E_INVALID and "brick_log2" in _lib.last_error()
    rc, dense = size(0, (5, 5, 5))                       # dense volumes ignore the shape
    assert rc == _lib.CLOUD_OK and dense == 32 * 20 * 9 * 2


def test_tune_keys_checked(lib):
    ok = lib.cloud_tune
    try:
        for key, good, bad in (("supertile", (-1, 0, 4, 64), (-2, 65)),
                               ("xcd_run", (-1, 0, 16, 65536), (-2, 65537)),
                               ("taa_tile", (16, 32, 64), (0, 8, 128)),
                               ("serve_blocks_per_cu", (0, 1, 4, 64), (-1, 65))):
            for v in good:
                assert ok(key.encode(), v) == _lib.CLOUD_OK, (key, v)
            for v in bad:
                assert ok(key.encode(), v) == _lib.CLOUD_E_INVALID, (key, v)
                assert key.encode() in _lib.load().cloud_last_error()
        assert ok(b"no_such_key", 1) == _lib.CLOUD_E_INVALID
        assert ok(None, 1) == _lib.CLOUD_E_INVALID
    finally:
        ok(b"supertile", -1)
        ok(b"xcd_run", -1)
        ok(b"taa_tile", 32)
        ok(b"serve_blocks_per_cu", 0)


def test_binding_checks_tensor_layout():
    import pytest
    import torch
    from paper_1609_05344_amd import _lib
    t = torch.zeros((4, 6, 4))
    assert _lib._ptr(t) == t.data_ptr() and _lib._ptr(None) == 0 and _lib._ptr(64) == 64
    with pytest.raises(ValueError, match="contiguous"):
        _lib._ptr(t.transpose(0, 1))
    assert _lib._out(t, (4, 6, 4), "cpu") is t
    with pytest.raises(ValueError, match="shape"):
        _lib._out(t, (6, 4, 4), "cpu")
    with pytest.raises(ValueError, match="float32"):
        _lib._out(t.to(torch.float16), (4, 6, 4), "cpu")
    assert _lib._out(None, (2, 3, 4), "cpu").shape == (2, 3, 4)


def test_binding_checks_images():
    import pytest
    import torch
    from paper_1609_05344_amd import _lib
    cur = torch.zeros((4, 6, 4))
    with pytest.raises(ValueError, match="history"):
        _lib.cloud_taa_resolve(cur, torch.zeros((6, 4, 4)), None, 0.1, 1)
    with pytest.raises(ValueError, match="current"):
        _lib.cloud_taa_resolve(cur.double(), None, None, 0.1, 0)
    with pytest.raises(ValueError, match="background"):
        _lib.cloud_composite(cur, torch.zeros((8, 12, 3)))


def test_binding_checks_rays():
    import pytest
    import torch
    from paper_1609_05344_amd import _lib
    o = torch.zeros((2, 3))
    with pytest.raises(ValueError, match="dirs"):
        _lib.cloud_march_rays(None, o, torch.zeros((2, 2)), None, None)
    with pytest.raises(ValueError, match="pixel_xy"):
        _lib.cloud_march_rays(None, o, o, torch.zeros((2, 2)), None)

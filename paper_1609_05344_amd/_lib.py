"""ctypes binding of libcloud.so: argument marshalling only.

Every function here mirrors one entry point of include/cloud.h under the same
name. Device buffers are torch tensors on a ROCm device (torch supplies device
memory and the current stream); all computation happens in the library's HIP
kernels. Loading fails loudly when the library has not been built.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_float, c_int, c_int32, c_int64, c_uint32, c_uint64, c_void_p

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcloud.so")

CLOUD_OK = 0
CLOUD_E_INVALID = -1
CLOUD_E_NOMEM = -2
CLOUD_E_HIP = -3
CLOUD_E_BUSY = -4
CLOUD_E_NOTFOUND = -5
CLOUD_E_CANCELLED = -6
CLOUD_F32, CLOUD_F16, CLOUD_BF16 = 0, 1, 2
DTYPES = {"f32": CLOUD_F32, "f16": CLOUD_F16, "bf16": CLOUD_BF16}


class CloudError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cloud error {code}: {msg}")
        self.code = code


class cloud_volume(ctypes.Structure):
    _fields_ = [
        ("base", c_void_p), ("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("dtype", c_int32),
        ("detail", c_void_p), ("dnx", c_int32), ("dny", c_int32), ("dnz", c_int32),
        ("ddtype", c_int32), ("detail_weight", c_float), ("detail_tiling", c_float),
        ("box_min", c_float * 3), ("box_max", c_float * 3), ("layout", c_int32),
    ]


class cloud_camera(ctypes.Structure):
    _fields_ = [("pos", c_float * 3), ("target", c_float * 3), ("up", c_float * 3),
                ("vfov_deg", c_float)]


class cloud_params(ctypes.Structure):
    _fields_ = [
        ("steps", c_int32), ("light_steps", c_int32), ("alpha", c_float), ("g", c_float),
        ("sun_dir", c_float * 3), ("sun_color", c_float * 3), ("ambient", c_float * 3),
        ("jitter", c_int32), ("seed", c_uint32), ("integration", c_int32), ("t_eps", c_float),
    ]


_lib = None


def load():
    """Load libcloud.so once; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1609_05344_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    lib.cloud_last_error.restype = c_char_p
    lib.cloud_last_error.argtypes = []
    lib.cloud_abi_version.restype = c_int
    lib.cloud_render.argtypes = [POINTER(cloud_volume), POINTER(cloud_camera), POINTER(cloud_params),
                                 c_uint32, c_int32, c_int32, c_void_p, c_void_p]
    lib.cloud_render_views.argtypes = [POINTER(cloud_volume), POINTER(cloud_camera), c_int32,
                                       POINTER(cloud_params), c_uint32, c_int32, c_int32,
                                       c_void_p, c_void_p]
    lib.cloud_march_rays.argtypes = [POINTER(cloud_volume), c_void_p, c_void_p, c_void_p, c_int64,
                                     POINTER(cloud_params), c_uint32, c_void_p, c_void_p]
    lib.cloud_taa_resolve.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_float,
                                      c_uint32, c_void_p]
    lib.cloud_jitter_offsets.argtypes = [c_void_p, c_int64, c_uint32, c_uint32, c_void_p, c_void_p]
    lib.cloud_check_buffer.argtypes = [c_void_p, c_uint64]
    for name in ("cloud_render", "cloud_render_views", "cloud_march_rays", "cloud_taa_resolve",
                 "cloud_jitter_offsets", "cloud_check_buffer"):
        getattr(lib, name).restype = c_int
    _lib = lib
    return lib


def last_error() -> str:
    return load().cloud_last_error().decode()


def check(rc: int) -> int:
    if rc != CLOUD_OK:
        raise CloudError(rc, last_error())
    return rc


# ---------------------------------------------------------------------------
# struct builders
# ---------------------------------------------------------------------------

def _ptr(t) -> int:
    if t is None:
        return 0
    if isinstance(t, int):
        return t
    return t.data_ptr()


def make_camera(cam) -> cloud_camera:
    c = cloud_camera()
    c.pos[:] = [float(x) for x in cam.pos]
    c.target[:] = [float(x) for x in cam.target]
    c.up[:] = [float(x) for x in cam.up]
    c.vfov_deg = float(cam.vfov_deg)
    return c


def make_params(p) -> cloud_params:
    c = cloud_params()
    c.steps, c.light_steps = int(p.steps), int(p.light_steps)
    c.alpha, c.g = float(p.alpha), float(p.g)
    c.sun_dir[:] = [float(x) for x in p.sun_dir]
    c.sun_color[:] = [float(x) for x in p.sun_color]
    c.ambient[:] = [float(x) for x in p.ambient]
    c.jitter, c.seed = int(p.jitter), int(p.seed) & 0xFFFFFFFF
    c.integration, c.t_eps = int(p.integration), float(p.t_eps)
    return c


class Volume:
    """Device density volume (plus optional detail) and its ABI descriptor.

    base / detail: ROCm tensors [nz][ny][nx] of float32, float16, bfloat16,
    or uint16 holding bfloat16 bit patterns (dtype="bf16")."""

    def __init__(self, base, detail=None, dtype: str | None = None, detail_weight: float = 0.3,
                 detail_tiling: float = 4.0, box_min=(-0.5, -0.5, -0.5), box_max=(0.5, 0.5, 0.5)):
        import torch
        self.base, self.detail = base, detail
        if dtype is None:
            dtype = {torch.float32: "f32", torch.float16: "f16", torch.bfloat16: "bf16",
                     torch.uint16: "bf16"}[base.dtype]
        self.dtype = dtype
        v = cloud_volume()
        v.base = _ptr(base)
        v.nz, v.ny, v.nx = (int(s) for s in base.shape)
        v.dtype = DTYPES[dtype]
        if detail is not None:
            v.detail = _ptr(detail)
            v.dnz, v.dny, v.dnx = (int(s) for s in detail.shape)
        v.ddtype = DTYPES[dtype]
        v.detail_weight, v.detail_tiling = float(detail_weight), float(detail_tiling)
        v.box_min[:] = [float(x) for x in box_min]
        v.box_max[:] = [float(x) for x in box_max]
        v.layout = 0
        self.struct = v


def _stream(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _out(out, shape, device):
    import torch
    if out is None:
        return torch.empty(shape, dtype=torch.float32, device=device)
    return out


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ---------------------------------------------------------------------------

def cloud_render(volume: Volume, camera, params, frame_index: int, width: int, height: int,
                 out=None, stream=None):
    out = _out(out, (height, width, 4), volume.base.device)
    cam, prm = make_camera(camera), make_params(params)
    check(load().cloud_render(ctypes.byref(volume.struct), ctypes.byref(cam), ctypes.byref(prm),
                              int(frame_index) & 0xFFFFFFFF, int(width), int(height), _ptr(out),
                              _stream(stream)))
    return out


def cloud_render_views(volume: Volume, cameras, params, frame_index: int, width: int, height: int,
                       out=None, stream=None):
    n = len(cameras)
    out = _out(out, (n, height, width, 4), volume.base.device)
    cams = (cloud_camera * max(n, 1))(*[make_camera(c) for c in cameras])
    prm = make_params(params)
    check(load().cloud_render_views(ctypes.byref(volume.struct), cams, n, ctypes.byref(prm),
                                    int(frame_index) & 0xFFFFFFFF, int(width), int(height),
                                    _ptr(out), _stream(stream)))
    return out


def cloud_march_rays(volume: Volume, origins, dirs, pixel_xy, params, frame_index: int = 0,
                     out=None, stream=None):
    n = int(origins.shape[0])
    out = _out(out, (n, 4), volume.base.device)
    prm = make_params(params)
    check(load().cloud_march_rays(ctypes.byref(volume.struct), _ptr(origins), _ptr(dirs),
                                  _ptr(pixel_xy), n, ctypes.byref(prm),
                                  int(frame_index) & 0xFFFFFFFF, _ptr(out), _stream(stream)))
    return out


def cloud_check_buffer(ptr, nbytes: int) -> int:
    """CLOUD_OK if [ptr, ptr + nbytes) lies inside one device allocation."""
    return load().cloud_check_buffer(_ptr(ptr), int(nbytes))


def cloud_jitter_offsets(pixel_xy, frame_index: int, seed: int, out=None, stream=None):
    import torch
    n = int(pixel_xy.shape[0])
    if out is None:
        out = torch.empty((n,), dtype=torch.int32, device=pixel_xy.device)
    check(load().cloud_jitter_offsets(_ptr(pixel_xy), n, int(frame_index) & 0xFFFFFFFF,
                                      int(seed) & 0xFFFFFFFF, _ptr(out), _stream(stream)))
    return out


def cloud_taa_resolve(current, history, out, blend: float, frame_index: int, stream=None):
    height, width = int(current.shape[0]), int(current.shape[1])
    if out is None:
        out = _out(None, (height, width, 4), current.device)
    check(load().cloud_taa_resolve(_ptr(current), _ptr(history), _ptr(out), width, height,
                                   float(blend), int(frame_index) & 0xFFFFFFFF, _stream(stream)))
    return out

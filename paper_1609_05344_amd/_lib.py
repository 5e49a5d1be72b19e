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
LAYOUTS = {"dense": 0, "quad": 1, "oct": 2}
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
        ("occupancy", c_void_p), ("occupancy_log2", c_int32), ("brick_log2", c_int32 * 3),
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


ABI_VERSION = 5   # the struct layouts and signatures this binding marshals


def load():
    """Load libcloud.so once; raises if it is missing or was built for
    another ABI version (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1609_05344_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    lib.cloud_last_error.restype = c_char_p
    lib.cloud_last_error.argtypes = []
    lib.cloud_abi_version.restype = c_int
    if lib.cloud_abi_version() != ABI_VERSION:
        raise RuntimeError(f"{LIB_PATH} has ABI version {lib.cloud_abi_version()}, this binding "
                           f"needs {ABI_VERSION}; rebuild with `python -m paper_1609_05344_amd.build`")
    lib.cloud_render.argtypes = [POINTER(cloud_volume), POINTER(cloud_camera), POINTER(cloud_params),
                                 c_uint32, c_int32, c_int32, c_void_p, c_void_p]
    lib.cloud_render_views.argtypes = [POINTER(cloud_volume), POINTER(cloud_camera), c_int32,
                                       POINTER(cloud_params), c_uint32, c_int32, c_int32,
                                       c_void_p, c_void_p]
    lib.cloud_march_rays.argtypes = [POINTER(cloud_volume), c_void_p, c_void_p, c_void_p, c_int64,
                                     POINTER(cloud_params), c_uint32, c_void_p, c_void_p]
    lib.cloud_taa_resolve.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_float,
                                      c_uint32, c_void_p]
    lib.cloud_render_resolve.argtypes = [POINTER(cloud_volume), POINTER(cloud_camera), c_int32,
                                         POINTER(cloud_params), c_uint32, c_int32, c_int32,
                                         c_void_p, c_void_p, c_void_p, c_void_p, c_float,
                                         c_uint32, c_void_p]
    lib.cloud_jitter_offsets.argtypes = [c_void_p, c_int64, c_uint32, c_uint32, c_void_p, c_void_p]
    lib.cloud_check_buffer.argtypes = [c_void_p, c_uint64]
    lib.cloud_tune.argtypes = [c_char_p, c_int32]
    lib.cloud_volume_occupancy_bytes.argtypes = [POINTER(cloud_volume), POINTER(c_uint64),
                                                 POINTER(c_int32)]
    lib.cloud_volume_occupancy.argtypes = [POINTER(cloud_volume), c_void_p, c_uint64,
                                           POINTER(cloud_volume), c_void_p]
    lib.cloud_volume_occupancy_bytes.restype = c_int
    lib.cloud_volume_occupancy.restype = c_int
    lib.cloud_count_lookups.argtypes = [POINTER(cloud_volume), POINTER(cloud_camera),
                                        POINTER(cloud_params), c_uint32, c_int32, c_int32,
                                        c_void_p, c_void_p]
    lib.cloud_render_depth.argtypes = [POINTER(cloud_volume), POINTER(cloud_camera),
                                       POINTER(cloud_params), c_uint32, c_int32, c_int32,
                                       c_void_p, c_void_p, c_void_p]
    lib.cloud_taa_resolve_reproject.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p,
                                                POINTER(cloud_camera), POINTER(cloud_camera),
                                                c_int32, c_int32, c_float, c_uint32, c_void_p]
    lib.cloud_composite.argtypes = [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_int32,
                                    c_int32, c_void_p]
    lib.cloud_lookup_trace.argtypes = [POINTER(cloud_volume), POINTER(cloud_camera), c_int32,
                                       POINTER(cloud_params), c_uint32, c_int32, c_int32,
                                       c_void_p, c_void_p]
    lib.cloud_gather_record.argtypes = [POINTER(cloud_volume), POINTER(cloud_camera), c_int32,
                                        POINTER(cloud_params), c_uint32, c_int32, c_int32,
                                        c_void_p, c_int32, c_void_p, c_void_p, c_void_p]
    lib.cloud_gather_replay.argtypes = [POINTER(cloud_volume), c_int32, c_int32, c_int32,
                                        c_void_p, c_int32, c_void_p, c_int32, c_int32, c_void_p,
                                        c_void_p]
    lib.cloud_volume_packed_bytes.argtypes = [POINTER(cloud_volume), c_int32, POINTER(c_uint64)]
    lib.cloud_volume_pack.argtypes = [POINTER(cloud_volume), c_int32, c_void_p, c_uint64,
                                      POINTER(cloud_volume), c_void_p]
    for name in ("cloud_render", "cloud_render_views", "cloud_march_rays", "cloud_taa_resolve",
                 "cloud_jitter_offsets", "cloud_check_buffer", "cloud_count_lookups",
                 "cloud_lookup_trace", "cloud_gather_record", "cloud_gather_replay",
                 "cloud_render_depth",
                 "cloud_taa_resolve_reproject", "cloud_composite",
                 "cloud_volume_packed_bytes", "cloud_volume_pack", "cloud_tune"):
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
    """Device address of a tensor (or a raw address, or 0 for None). The
    library reads and writes dense row-major arrays, so a tensor must be
    contiguous."""
    if t is None:
        return 0
    if isinstance(t, int):
        return t
    if not t.is_contiguous():
        raise ValueError(f"tensor of shape {tuple(t.shape)} is not contiguous")
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
    """A float32 output of the given shape: `out` when given (checked), else
    a new tensor on `device`."""
    import torch
    if out is None:
        return torch.empty(shape, dtype=torch.float32, device=device)
    if out.dtype != torch.float32 or tuple(out.shape) != tuple(shape):
        raise ValueError(f"out must be float32 of shape {tuple(shape)}, "
                         f"not {out.dtype} of shape {tuple(out.shape)}")
    return out


def _image(t, shape, what):
    """Check an input image (None passes: the library decides whether it may
    be absent)."""
    import torch
    if t is not None and (t.dtype != torch.float32 or tuple(t.shape) != tuple(shape)):
        raise ValueError(f"{what} must be float32 of shape {tuple(shape)}, "
                         f"not {t.dtype} of shape {tuple(t.shape)}")
    return t


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
    import torch
    n = int(origins.shape[0])
    _image(origins, (n, 3), "origins")
    _image(dirs, (n, 3), "dirs")
    if pixel_xy is not None and (pixel_xy.dtype not in (torch.int32, torch.uint32)
                                 or tuple(pixel_xy.shape) != (n, 2)):
        raise ValueError(f"pixel_xy must be 32-bit integers of shape ({n}, 2)")
    out = _out(out, (n, 4), volume.base.device)
    prm = make_params(params)
    check(load().cloud_march_rays(ctypes.byref(volume.struct), _ptr(origins), _ptr(dirs),
                                  _ptr(pixel_xy), n, ctypes.byref(prm),
                                  int(frame_index) & 0xFFFFFFFF, _ptr(out), _stream(stream)))
    return out


def cloud_count_lookups(volume: Volume, camera, params, frame_index: int, width: int,
                        height: int, out=None, stream=None):
    """Density lookups a render of this frame performs (device int64 tensor [1],
    accumulated into `out` when given)."""
    import torch
    if out is None:
        out = torch.zeros((1,), dtype=torch.int64, device=volume.base.device)
    cam, prm = make_camera(camera), make_params(params)
    check(load().cloud_count_lookups(ctypes.byref(volume.struct), ctypes.byref(cam),
                                     ctypes.byref(prm), int(frame_index) & 0xFFFFFFFF, int(width),
                                     int(height), _ptr(out), _stream(stream)))
    return out


def cloud_render_depth(volume: Volume, camera, params, frame_index: int, width: int, height: int,
                       out=None, depth=None, stream=None):
    """cloud_render plus the representative depth; returns (rgba [H,W,4],
    depth [H,W])."""
    import torch
    out = _out(out, (height, width, 4), volume.base.device)
    if depth is None:
        depth = torch.empty((height, width), dtype=torch.float32, device=volume.base.device)
    _image(depth, (height, width), "depth")
    cam, prm = make_camera(camera), make_params(params)
    check(load().cloud_render_depth(ctypes.byref(volume.struct), ctypes.byref(cam),
                                    ctypes.byref(prm), int(frame_index) & 0xFFFFFFFF, int(width),
                                    int(height), _ptr(out), _ptr(depth), _stream(stream)))
    return out, depth


def cloud_taa_resolve_reproject(current, depth, history, out, camera, prev_camera, blend: float,
                                frame_index: int, stream=None):
    """Reprojected temporal resolve into `out` (which must not alias the
    inputs); returns out."""
    H, W = int(current.shape[0]), int(current.shape[1])
    _image(current, (H, W, 4), "current")
    _image(depth, (H, W), "depth")
    _image(history, (H, W, 4), "history")
    out = _out(out, (H, W, 4), current.device)
    cam, prev = make_camera(camera), make_camera(prev_camera)
    check(load().cloud_taa_resolve_reproject(_ptr(current), _ptr(depth), _ptr(history), _ptr(out),
                                             ctypes.byref(cam), ctypes.byref(prev), W, H,
                                             float(blend), int(frame_index) & 0xFFFFFFFF,
                                             _stream(stream)))
    return out


def cloud_composite(cloud, background, out=None, stream=None):
    """Up-sample the cloud layer [h, w, 4] to the background's size and
    composite it over the background; returns out [H, W, 4]."""
    lh, lw = int(cloud.shape[0]), int(cloud.shape[1])
    H, W = int(background.shape[0]), int(background.shape[1])
    _image(cloud, (lh, lw, 4), "cloud")
    _image(background, (H, W, 4), "background")
    out = _out(out, (H, W, 4), background.device)
    check(load().cloud_composite(_ptr(cloud), lw, lh, _ptr(background), _ptr(out), W, H,
                                 _stream(stream)))
    return out


def cloud_lookup_trace(volume: Volume, cameras, params, frame_index: int, width: int, height: int,
                       out=None, stream=None):
    """Per-pixel (primary samples, light-march mask) of a render of these views:
    device int32 tensor [n_views, H, W, 2] (the bits are uint32)."""
    import torch
    n = len(cameras)
    if out is None:
        out = torch.empty((n, height, width, 2), dtype=torch.int32, device=volume.base.device)
    cams = (cloud_camera * max(n, 1))(*[make_camera(c) for c in cameras])
    prm = make_params(params)
    check(load().cloud_lookup_trace(ctypes.byref(volume.struct), cams, n, ctypes.byref(prm),
                                    int(frame_index) & 0xFFFFFFFF, int(width), int(height),
                                    _ptr(out), _stream(stream)))
    return out


def gather_waves(n_views: int, width: int, height: int) -> int:
    """Wavefronts of a render of n_views width x height views (four per 16x16 tile)."""
    return n_views * ((width + 15) // 16) * ((height + 15) // 16) * 4


def cloud_gather_record(volume: Volume, cameras, params, frame_index: int, width: int,
                        height: int, trace, max_slots: int = 0, codes=None, slot_counts=None,
                        stream=None):
    """The render's lookups as per-wavefront slots of corner codes; returns
    (codes [n_waves, max_slots, 64] int32 (uint32 bits), slot_counts [n_waves]
    int32). max_slots 0: steps * (1 + light_steps)."""
    import torch
    n = len(cameras)
    if max_slots <= 0:
        max_slots = int(params.steps) * (1 + int(params.light_steps))
    waves = gather_waves(n, width, height)
    dev = volume.base.device
    if codes is None:
        codes = torch.empty((waves, max_slots, 64), dtype=torch.int32, device=dev)
    if slot_counts is None:
        slot_counts = torch.empty((waves,), dtype=torch.int32, device=dev)
    cams = (cloud_camera * max(n, 1))(*[make_camera(c) for c in cameras])
    prm = make_params(params)
    check(load().cloud_gather_record(ctypes.byref(volume.struct), cams, n, ctypes.byref(prm),
                                     int(frame_index) & 0xFFFFFFFF, int(width), int(height),
                                     _ptr(trace), int(max_slots), _ptr(codes), _ptr(slot_counts),
                                     _stream(stream)))
    return codes, slot_counts


def cloud_gather_replay(volume: Volume, n_views: int, width: int, height: int, codes,
                        slot_counts, mode: int = 0, blocks_per_cu: int = 0, out=None,
                        stream=None):
    """Fetch-only replay of recorded slots (mode 0) or of as many uniformly
    random corners (mode 1); returns the [n_waves, 64] int32 XOR output."""
    import torch
    waves = gather_waves(n_views, width, height)
    max_slots = int(codes.shape[1]) if codes.dim() == 3 else int(codes.numel() // (waves * 64))
    if out is None:
        out = torch.empty((waves, 64), dtype=torch.int32, device=volume.base.device)
    check(load().cloud_gather_replay(ctypes.byref(volume.struct), int(n_views), int(width),
                                     int(height), _ptr(codes), max_slots, _ptr(slot_counts),
                                     int(mode), int(blocks_per_cu), _ptr(out), _stream(stream)))
    return out


def _struct_with_brick(volume: Volume, brick):
    st = cloud_volume()
    ctypes.memmove(ctypes.byref(st), ctypes.byref(volume.struct), ctypes.sizeof(cloud_volume))
    if brick is not None:
        st.brick_log2[:] = [int(b) for b in brick]
    return st


def cloud_volume_packed_bytes(volume: Volume, layout: str, brick=None) -> int:
    """Bytes of a packed copy; brick: (bx, by, bz) log2 brick shape, or None
    for the default."""
    n = c_uint64(0)
    st = _struct_with_brick(volume, brick)
    check(load().cloud_volume_packed_bytes(ctypes.byref(st), LAYOUTS[layout], ctypes.byref(n)))
    return int(n.value)


def cloud_volume_pack(volume: Volume, layout: str, stream=None, brick=None) -> "Volume":
    """Packed copy of a dense volume (a new device buffer owned by the returned
    Volume); brick: (bx, by, bz) log2 brick shape of the packed entries, or
    None for the default (1, 1, 1)."""
    import torch
    nbytes = cloud_volume_packed_bytes(volume, layout, brick)
    buf = torch.empty((nbytes,), dtype=torch.uint8, device=volume.base.device)
    packed = cloud_volume()
    st = _struct_with_brick(volume, brick)
    check(load().cloud_volume_pack(ctypes.byref(st), LAYOUTS[layout], _ptr(buf), nbytes,
                                   ctypes.byref(packed), _stream(stream)))
    out = Volume.__new__(Volume)
    out.base, out.detail, out.dtype = buf, volume.detail, volume.dtype
    out.dense = volume
    out.occupancy = getattr(volume, "occupancy", None)
    out.struct = packed
    return out


def cloud_volume_occupancy(volume: Volume, stream=None) -> "Volume":
    """The same (dense) volume with an occupancy bitmap attached (a new device
    buffer owned by the returned Volume); pack it afterwards to keep both."""
    import torch
    nbytes, lg = c_uint64(0), c_int32(0)
    check(load().cloud_volume_occupancy_bytes(ctypes.byref(volume.struct), ctypes.byref(nbytes),
                                              ctypes.byref(lg)))
    buf = torch.empty((max(int(nbytes.value) // 4, 1),), dtype=torch.int32, device=volume.base.device)
    withocc = cloud_volume()
    check(load().cloud_volume_occupancy(ctypes.byref(volume.struct), _ptr(buf), int(nbytes.value),
                                        ctypes.byref(withocc), _stream(stream)))
    out = Volume.__new__(Volume)
    out.base, out.detail, out.dtype = volume.base, volume.detail, volume.dtype
    out.dense = volume
    out.occupancy = buf
    out.struct = withocc
    return out


def cloud_tune(key: str, value: int) -> None:
    check(load().cloud_tune(key.encode(), int(value)))


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
    _image(current, (height, width, 4), "current")
    _image(history, (height, width, 4), "history")
    out = _out(out, (height, width, 4), current.device)
    check(load().cloud_taa_resolve(_ptr(current), _ptr(history), _ptr(out), width, height,
                                   float(blend), int(frame_index) & 0xFFFFFFFF, _stream(stream)))
    return out


def cloud_render_resolve(volume: Volume, camera, params, frame_index: int, width: int,
                         height: int, prev, history, resolved, blend: float,
                         prev_frame_index: int, out=None, stream=None):
    """The render of frame_index into `out` and the resolve of `prev` (the
    previous frame's render) against `history` into `resolved`, in one launch;
    returns (out, resolved). `camera` is one camera ([H, W, 4] images) or a
    list of them ([n, H, W, 4] images, as cloud_render_views)."""
    cams = list(camera) if isinstance(camera, (list, tuple)) else [camera]
    shape = (len(cams), height, width, 4) if isinstance(camera, (list, tuple)) else (height, width, 4)
    _image(prev, shape, "prev")
    _image(history, shape, "history")
    out = _out(out, shape, volume.base.device)
    resolved = _out(resolved, shape, volume.base.device)
    arr = (cloud_camera * max(len(cams), 1))(*[make_camera(c) for c in cams])
    prm = make_params(params)
    check(load().cloud_render_resolve(ctypes.byref(volume.struct), arr, len(cams),
                                      ctypes.byref(prm), int(frame_index) & 0xFFFFFFFF,
                                      int(width), int(height), _ptr(out), _ptr(prev),
                                      _ptr(history), _ptr(resolved), float(blend),
                                      int(prev_frame_index) & 0xFFFFFFFF, _stream(stream)))
    return out, resolved


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------

class cloud_serve_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", c_uint64), ("max_batch", c_int32), ("max_queue", c_int32),
                ("device", c_int32), ("taa_blend", c_float), ("use_graphs", c_int32),
                ("queues", c_int32), ("history_in_output", c_int32), ("start_lead_us", c_int32)]


class cloud_serve_stats_t(ctypes.Structure):
    _fields_ = [(n, c_uint64) for n in ("queued", "admitted", "running", "completed", "rejected",
                                        "cancelled", "failed", "streams", "bytes_in_use",
                                        "batches")]


class cloud_completion(ctypes.Structure):
    _fields_ = [("request_id", c_uint64), ("stream_id", c_uint64), ("status", c_int32),
                ("reserved", c_int32), ("t_submit_ns", c_int64), ("t_admit_ns", c_int64),
                ("t_start_ns", c_int64), ("t_done_ns", c_int64)]


def _bind_serve(lib):
    if getattr(lib, "_serve_bound", False):
        return lib
    lib.cloud_serve_create.argtypes = [POINTER(cloud_volume), POINTER(cloud_serve_config),
                                       POINTER(c_void_p)]
    lib.cloud_serve_submit.argtypes = [c_void_p, c_uint64, POINTER(cloud_camera),
                                       POINTER(cloud_params), c_int32, c_int32, c_uint32, c_void_p,
                                       POINTER(c_uint64)]
    lib.cloud_serve_poll.argtypes = [c_void_p, POINTER(cloud_completion), c_int32, POINTER(c_int32)]
    lib.cloud_serve_wait.argtypes = [c_void_p, c_int64]
    lib.cloud_serve_stats.argtypes = [c_void_p, POINTER(cloud_serve_stats_t)]
    lib.cloud_serve_close_stream.argtypes = [c_void_p, c_uint64]
    lib.cloud_serve_destroy.argtypes = [c_void_p]
    for n in ("cloud_serve_create", "cloud_serve_submit", "cloud_serve_poll", "cloud_serve_wait",
              "cloud_serve_stats", "cloud_serve_close_stream", "cloud_serve_destroy"):
        getattr(lib, n).restype = c_int
    lib._serve_bound = True
    return lib


class Server:
    """cloud_serve_* over one shared Volume. Keeps the Volume alive."""

    def __init__(self, volume: Volume, budget_bytes: int = 64 << 30, max_batch: int = 64,
                 max_queue: int = 1024, device: int = 0, taa_blend: float = 0.1,
                 use_graphs: bool = True, queues: int = 1, history_in_output: bool = False,
                 start_lead_us: int = 0):
        self.lib = _bind_serve(load())
        self.volume = volume
        cfg = cloud_serve_config(int(budget_bytes), int(max_batch), int(max_queue), int(device),
                                 float(taa_blend), 1 if use_graphs else 0, int(queues),
                                 1 if history_in_output else 0, int(start_lead_us))
        h = c_void_p()
        check(self.lib.cloud_serve_create(ctypes.byref(volume.struct), ctypes.byref(cfg),
                                          ctypes.byref(h)))
        self.handle = h

    def cloud_serve_submit(self, stream_id: int, camera, params, width: int, height: int,
                           frame_index: int, out) -> int:
        rid = c_uint64(0)
        cam, prm = make_camera(camera), make_params(params)
        rc = self.lib.cloud_serve_submit(self.handle, int(stream_id), ctypes.byref(cam),
                                         ctypes.byref(prm), int(width), int(height),
                                         int(frame_index) & 0xFFFFFFFF, _ptr(out),
                                         ctypes.byref(rid))
        check(rc)
        return int(rid.value)

    submit = cloud_serve_submit

    def try_submit(self, *args):
        """Like submit, but returns the CLOUD_E_* code instead of raising."""
        rid = c_uint64(0)
        stream_id, camera, params, width, height, frame_index, out = args
        cam, prm = make_camera(camera), make_params(params)
        rc = self.lib.cloud_serve_submit(self.handle, int(stream_id), ctypes.byref(cam),
                                         ctypes.byref(prm), int(width), int(height),
                                         int(frame_index) & 0xFFFFFFFF, _ptr(out),
                                         ctypes.byref(rid))
        return rc, int(rid.value)

    def cloud_serve_poll(self, max_items: int = 256):
        arr = (cloud_completion * max(max_items, 1))()
        n = c_int32(0)
        check(self.lib.cloud_serve_poll(self.handle, arr, int(max_items), ctypes.byref(n)))
        return [{"request_id": int(c.request_id), "stream_id": int(c.stream_id),
                 "status": int(c.status), "t_submit_ns": int(c.t_submit_ns),
                 "t_admit_ns": int(c.t_admit_ns), "t_start_ns": int(c.t_start_ns),
                 "t_done_ns": int(c.t_done_ns)} for c in arr[:n.value]]

    poll = cloud_serve_poll

    def cloud_serve_wait(self, timeout_s: float) -> bool:
        rc = self.lib.cloud_serve_wait(self.handle, int(timeout_s * 1e9))
        if rc < 0:
            check(rc)
        return rc == 1

    wait = cloud_serve_wait

    def cloud_serve_stats(self) -> dict:
        s = cloud_serve_stats_t()
        check(self.lib.cloud_serve_stats(self.handle, ctypes.byref(s)))
        return {n: int(getattr(s, n)) for n, _ in cloud_serve_stats_t._fields_}

    stats = cloud_serve_stats

    def cloud_serve_close_stream(self, stream_id: int) -> int:
        return self.lib.cloud_serve_close_stream(self.handle, int(stream_id))

    close_stream = cloud_serve_close_stream

    def cloud_serve_destroy(self):
        if self.handle is not None and self.handle.value:
            check(self.lib.cloud_serve_destroy(self.handle))
        self.handle = None

    destroy = cloud_serve_destroy

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

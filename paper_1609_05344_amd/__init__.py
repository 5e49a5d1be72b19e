"""MI355X (gfx950) cloud raymarch: the method of "Optimisations for Real-Time
Volumetric Cloudscapes" (Toft, Bowles and Zimmermann, arXiv 1609.05344) as
hand-written HIP kernels behind a C ABI (include/cloud.h).

The Python layer is a thin ctypes binding (argument marshalling only); the
library is loaded on first use and raises if it has not been built.
"""

from ._lib import (  # noqa: F401
    CloudError,
    Server,
    Volume,
    cloud_check_buffer,
    cloud_count_lookups,
    cloud_lookup_trace,
    cloud_gather_record,
    cloud_gather_replay,
    gather_waves,
    cloud_jitter_offsets,
    cloud_march_rays,
    cloud_render,
    cloud_render_views,
    cloud_render_depth,
    cloud_render_resolve,
    cloud_taa_resolve_reproject,
    cloud_composite,
    cloud_taa_resolve,
    cloud_tune,
    cloud_volume_occupancy,
    cloud_volume_pack,
    cloud_volume_packed_bytes,
    last_error,
    load,
)


def device_volume(scene, device="cuda", layout: str = "dense", occupancy: bool = False,
                  brick=None):
    """Upload a seeded scene's stored volumes (see scenes.make_scene),
    optionally with an occupancy bitmap and in a packed layout (entries in
    bricks of shape `brick`, log2 per axis; None for the default)."""
    import numpy as np
    import torch

    w = scene.workload

    def up(a):
        if a is None:
            return None
        if a.dtype == np.uint16:   # bfloat16 bit patterns
            return torch.from_numpy(a.view(np.int16)).to(device).view(torch.bfloat16)
        return torch.from_numpy(np.ascontiguousarray(a)).to(device)

    base, det = up(scene.base_stored), up(scene.detail_stored)
    dtype = {np.dtype(np.float32): "f32", np.dtype(np.float16): "f16",
             np.dtype(np.uint16): "bf16"}[scene.base_stored.dtype]
    vol = Volume(base, det, dtype=dtype, detail_weight=w.params.detail_weight,
                 detail_tiling=w.params.detail_tiling)
    if occupancy:
        vol = cloud_volume_occupancy(vol)
    if layout != "dense":
        vol = cloud_volume_pack(vol, layout, brick=brick)
    return vol

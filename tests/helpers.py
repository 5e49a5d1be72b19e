"""Shared test plumbing: seeded scenes for both sides, device upload, and
error summaries. Holds none of the method's arithmetic."""

import numpy as np

from oracle import cloud as O
from paper_1609_05344_amd import scenes

FP32_TOL = 1e-4     # max-abs RGBA, float32 storage and arithmetic
HALF_TOL = 2e-3     # max-abs RGBA, 16-bit storage, against the decoded volume


def oracle_volume(scene):
    w = scene.workload
    return O.OracleVolume(base=scene.base_f64, detail=scene.detail_f64,
                          detail_weight=w.params.detail_weight,
                          detail_tiling=w.params.detail_tiling)


def const_scene(c, n=8, dtype="f32"):
    """A homogeneous volume wrapped as a scene."""
    w = scenes.workload("C1")
    base = scenes.quantise(np.full((n, n, n), float(c)), dtype)
    return scenes.Scene(w, base, scenes.decode(base, dtype))


def max_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    assert a.shape == b.shape, (a.shape, b.shape)
    return float(np.max(np.abs(a - b))) if a.size else 0.0


def to_np(t):
    return t.detach().cpu().numpy()

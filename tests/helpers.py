"""Shared test plumbing: seeded scenes for both sides, device upload, error
summaries, and the oracle's resolve chain at sampled pixels (its steps are
the oracle's own render and resolve). Holds none of the method's arithmetic."""

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


def oracle_chain_sampled(ovol, cams, params, W, H, frames, pix, blend=0.1):
    """The oracle's render + resolve chain at pixels pix [n, 2] (px, py):
    per frame, (current frame, resolved output) at those pixels, [n, 4] each.
    A resolved pixel depends each frame only on the current frame's 3x3
    neighbourhood (edge-clamped) and its own history, so per frame the oracle
    renders just those neighbourhoods and resolves each sampled pixel from
    its own patch. The first frame has no history and is copied."""
    n = len(pix)
    offs = [(dx, dy) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    nb = np.stack([np.stack([np.clip(pix[:, 0] + dx, 0, W - 1),
                             np.clip(pix[:, 1] + dy, 0, H - 1)], 1) for dx, dy in offs], 1)
    uniq, inv = np.unique(nb.reshape(-1, 2), axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    hist, out = None, []
    for k, f in enumerate(frames):
        vals = O.render(ovol, cams[k], params, W, H, frame=f, pixels=uniq)
        patch = vals[inv].reshape(n, 3, 3, 4)
        # the patches side by side: patch i is columns 3i..3i+2 of a 3-row
        # image, so the centre (1, 3i+1) sees exactly its own neighbourhood
        img = patch.transpose(1, 0, 2, 3).reshape(3, 3 * n, 4)
        himg = None
        if hist is not None:
            himg = np.zeros_like(img)
            himg[1, 1::3] = hist
        res = O.taa_resolve(img, himg, blend, 0 if k == 0 else f)
        hist = res[1, 1::3].copy()
        out.append((patch[:, 1, 1].copy(), hist))
    return out

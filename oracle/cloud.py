"""FP64 oracle: the cloud raymarch step by step (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
use this module. It is written for a reader to check against the paper by eye:
numpy arrays in float64, one loop over the primary steps, no blocking or
fusion beyond what the method states.

Readings taken where the paper is silent or garbled (each one is repeated at
the function that applies it):

* R1  The lighting term L of the analytic integral carries the scattering
      coefficient rho*alpha (albedo 1), so one step contributes
      T0 * L_in * (1 - exp(-rho*alpha*D)).
* R2  The integral's last line is evaluated at x = D.
* R3  The naive rule S = T L is a Riemann sum: after T is updated,
      S += T * rho*alpha*D * L_in.
* R4  alpha is the extinction per unit density; scattering equals extinction.
* R5  "transmittance" is the transmitted fraction; alpha (opacity) = 1 - T.
* R6  A fixed number N of samples over the ray's chord through the box;
      sample i sits at t_near + (i + j) D with one per-pixel offset j in [0, 1);
      without jitter j = 0.5.
* R7  The light march goes to the box exit along the sun direction in L equal
      steps sampled at their midpoints, and is skipped where rho = 0.
* R8  Henyey-Greenstein with mu = dot(view direction, direction to the sun),
      normalised over the sphere.
* R10 Texel centres at (k + 0.5)/n, clamp-to-edge for the base volume,
      repeat for the detail volume, lerps in x, then y, then z as a + w (b - a).
* R11 Detail erosion rho = clamp((b - w_e d) / (1 - w_e d), 0, 1).
* R12 The march ending once the accumulated alpha is full is T < t_eps after
      the step's update.
* R13 Temporal resolve: per-channel 3x3 min/max clamp of the history, then
      out = h + beta (cur - h); frame 0 (or no history) copies the current frame.
* R14 The random offset is a PCG hash chain (Jarzynski and Olano 2020) of the
      pixel, frame and seed, so the library and the oracle draw the same j.
* R16 Pinhole camera, vertical field of view, pixel centres, row 0 at the top.
* R17 Coherent jitter variants (Section 5 leaves cheaper jitter to future
      work; Section 4 reports that one offset for every ray of a frame
      removes the cost but defeats the resolve): one offset per 8x8-pixel
      tile (the hash of (px >> 3, py >> 3)) and one per frame (of (0, 0)).
* R18 Reprojected resolve (Playdead's TAA, Section 3.2, reprojects its
      history): a ray's representative depth is its mean sample distance
      weighted by the opacity each step adds, where alpha >= 0.01; the middle
      of its chord through the box below that; at infinity for a miss. The
      point there is projected into the previous camera, the history sampled
      bilinearly (edge clamp), then clamped and blended as in R13; a point
      behind the previous camera or off its image takes the current value.
* R19 Composite (Section 3.2): the resolved low-resolution layer is
      up-sampled bilinearly with pixel centres aligned (edge clamp) and laid
      over the scene with the premultiplied over operator.
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_M32 = 0xFFFFFFFF


# ---------------------------------------------------------------------------
# Jitter: PCG hash (R14; Section 3.2 asks for a per-pixel random start offset)
# ---------------------------------------------------------------------------

def pcg_hash(v):
    """PCG-RXS-M-XS 32-bit hash of Jarzynski and Olano (JCGT 2020), mod 2^32.

    Works on Python ints or numpy uint32 arrays."""
    if isinstance(v, np.ndarray):
        v = v.astype(np.uint64) & _M32
        s = (v * 747796405 + 2891336453) & _M32
        w = (((s >> ((s >> 28) + 4)) ^ s) * 277803737) & _M32
        return ((w >> 22) ^ w).astype(np.uint32)
    v = int(v) & _M32
    s = (v * 747796405 + 2891336453) & _M32
    w = (((s >> ((s >> 28) + 4)) ^ s) * 277803737) & _M32
    return ((w >> 22) ^ w) & _M32


def jitter_offset(px, py, frame: int, seed: int):
    """Per-pixel start offset j in [0, 1 - 2^-24] (Section 3.2, reading R14).

    h = pcg(px + pcg(py + pcg(frame + pcg(seed)))), additions mod 2^32;
    j = (h >> 8) * 2^-24, exact in both float32 and float64."""
    hs = pcg_hash(int(seed))
    hf = pcg_hash((int(frame) + hs) & _M32)
    if isinstance(px, np.ndarray) or isinstance(py, np.ndarray):
        px = np.asarray(px).astype(np.uint64)
        py = np.asarray(py).astype(np.uint64)
        hy = pcg_hash((py + hf) & _M32)
        h = pcg_hash((px + hy.astype(np.uint64)) & _M32)
        return (h >> 8).astype(np.float64) * 2.0 ** -24
    hy = pcg_hash((int(py) + hf) & _M32)
    h = pcg_hash((int(px) + hy) & _M32)
    return (h >> 8) * 2.0 ** -24


JITTER_NONE, JITTER_PIXEL, JITTER_TILE, JITTER_FRAME = 0, 1, 2, 3


def jitter_for(mode: int, px, py, frame: int, seed: int):
    """Start offsets of pixels (px, py) under a jitter mode (reading R17).

    0: none (None: the march uses j = 0.5); 1: per pixel (Section 3.2), the
    hash of (px, py); 2: one offset per 8x8-pixel tile, the hash of
    (px >> 3, py >> 3); 3: one offset per frame, the hash of (0, 0). Modes 2
    and 3 are the coherent variants the paper's Section 5 points to."""
    mode = int(mode)
    if mode == JITTER_NONE:
        return None
    if mode not in (JITTER_PIXEL, JITTER_TILE, JITTER_FRAME):
        raise ValueError(f"unknown jitter mode {mode}")
    if np.ndim(px) == 0 and np.ndim(py) == 0:
        px, py = int(px), int(py)
    else:
        px = np.asarray(px, dtype=np.int64)
        py = np.asarray(py, dtype=np.int64)
    if mode == JITTER_TILE:
        px, py = px >> 3, py >> 3
    elif mode == JITTER_FRAME:
        px, py = px * 0, py * 0
    return jitter_offset(px, py, frame, seed)


# ---------------------------------------------------------------------------
# Phase function (Section 1, Henyey-Greenstein; reading R8)
# ---------------------------------------------------------------------------

def hg_phase(mu, g: float):
    """Henyey-Greenstein phase (1 - g^2) / (4 pi (1 + g^2 - 2 g mu)^(3/2))."""
    return (1.0 - g * g) / (4.0 * math.pi * (1.0 + g * g - 2.0 * g * np.asarray(mu, dtype=np.float64)) ** 1.5)


# ---------------------------------------------------------------------------
# Rays (Section 1: one ray per pixel into the volume; reading R16)
# ---------------------------------------------------------------------------

def _normalize(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.sqrt(np.sum(v * v, axis=-1, keepdims=True))


def camera_rays(cam, width: int, height: int, px, py):
    """Pinhole rays through pixel centres; returns (origins [n,3], unit dirs [n,3])."""
    pos = np.asarray(cam.pos, dtype=np.float64)
    f = _normalize(np.asarray(cam.target, dtype=np.float64) - pos)
    r = _normalize(np.cross(f, np.asarray(cam.up, dtype=np.float64)))
    u = np.cross(r, f)
    tan_half = math.tan(math.radians(cam.vfov_deg) * 0.5)
    px = np.asarray(px, dtype=np.float64)
    py = np.asarray(py, dtype=np.float64)
    x = (2.0 * (px + 0.5) / width - 1.0) * tan_half * (width / height)
    y = (1.0 - 2.0 * (py + 0.5) / height) * tan_half
    d = f[None, :] + x[:, None] * r[None, :] + y[:, None] * u[None, :]
    d = _normalize(d)
    o = np.broadcast_to(pos, d.shape).copy()
    return o, d


def ray_box(o, d, box_min, box_max):
    """Slab test; returns (t_near, t_far, hit) with t_near clamped at 0.

    An axis with d_k = 0 passes when box_min_k <= o_k <= box_max_k and fails
    otherwise. The ray misses when t_far <= t_near (Section 1: the march ends
    where the ray leaves the volume)."""
    o = np.asarray(o, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    n = o.shape[0]
    tn = np.zeros(n)
    tf = np.full(n, np.inf)
    ok = np.ones(n, dtype=bool)
    for k in range(3):
        dk, ok_ = d[:, k], o[:, k]
        par = dk == 0.0
        inside = (ok_ >= box_min[k]) & (ok_ <= box_max[k])
        ok &= ~par | inside
        with np.errstate(divide="ignore", invalid="ignore"):
            t0 = (box_min[k] - ok_) / dk
            t1 = (box_max[k] - ok_) / dk
        lo = np.where(par, -np.inf, np.minimum(t0, t1))
        hi = np.where(par, np.inf, np.maximum(t0, t1))
        tn = np.maximum(tn, lo)
        tf = np.minimum(tf, hi)
    hit = ok & (tf > tn)
    return tn, tf, hit


# ---------------------------------------------------------------------------
# Density (Section 1: the density is sampled at each step; readings R10, R11)
# ---------------------------------------------------------------------------

@dataclass
class OracleVolume:
    base: np.ndarray                      # float64 [nz][ny][nx], decoded exactly
    detail: Optional[np.ndarray] = None   # float64 [dz][dy][dx] or None
    detail_weight: float = 0.3
    detail_tiling: float = 4.0
    box_min: Sequence[float] = (-0.5, -0.5, -0.5)
    box_max: Sequence[float] = (0.5, 0.5, 0.5)


def _lerp(a, b, w):
    return a + w * (b - a)


def _trilinear(vol: np.ndarray, fx, fy, fz, repeat: bool):
    """Trilinear interpolation at continuous texel coordinates f (texel k's
    centre is at f = k); x, then y, then z."""
    nz, ny, nx = vol.shape
    flat = vol.reshape(-1)
    out = []
    for f, n in ((fx, nx), (fy, ny), (fz, nz)):
        k0 = np.floor(f)
        w = f - k0
        k0 = k0.astype(np.int64)
        k1 = k0 + 1
        if repeat:
            k0, k1 = np.mod(k0, n), np.mod(k1, n)
        else:
            k0, k1 = np.clip(k0, 0, n - 1), np.clip(k1, 0, n - 1)
        out.append((k0, k1, w))
    (x0, x1, wx), (y0, y1, wy), (z0, z1, wz) = out

    def at(z, y, x):
        return flat[(z * ny + y) * nx + x]

    c00 = _lerp(at(z0, y0, x0), at(z0, y0, x1), wx)
    c10 = _lerp(at(z0, y1, x0), at(z0, y1, x1), wx)
    c01 = _lerp(at(z1, y0, x0), at(z1, y0, x1), wx)
    c11 = _lerp(at(z1, y1, x0), at(z1, y1, x1), wx)
    return _lerp(_lerp(c00, c10, wy), _lerp(c01, c11, wy), wz)


def density(vol: OracleVolume, p):
    """Density at world points p [n,3] (R10 base lookup, R11 detail erosion)."""
    p = np.asarray(p, dtype=np.float64)
    bmin = np.asarray(vol.box_min, dtype=np.float64)
    bmax = np.asarray(vol.box_max, dtype=np.float64)
    uvw = (p - bmin) / (bmax - bmin)
    nz, ny, nx = vol.base.shape
    b = _trilinear(vol.base, uvw[:, 0] * nx - 0.5, uvw[:, 1] * ny - 0.5,
                   uvw[:, 2] * nz - 0.5, repeat=False)
    if vol.detail is None:
        return b
    dz, dy, dx = vol.detail.shape
    t = vol.detail_tiling
    d = _trilinear(vol.detail, uvw[:, 0] * t * dx - 0.5, uvw[:, 1] * t * dy - 0.5,
                   uvw[:, 2] * t * dz - 0.5, repeat=True)
    we = vol.detail_weight
    return np.clip((b - we * d) / (1.0 - we * d), 0.0, 1.0)


def light_transmittance(vol: OracleVolume, p, s_hat, light_steps: int, alpha: float):
    """Transmittance from p towards the sun (Section 1, Beer-Lambert; R7).

    Marches to the box exit along s_hat in light_steps equal steps sampled at
    their midpoints: T_L = exp(-alpha * d_l * sum_k rho(p + (k + 1/2) d_l s))."""
    p = np.asarray(p, dtype=np.float64)
    n = p.shape[0]
    if light_steps <= 0 or n == 0:
        return np.ones(n)
    tx = np.full(n, np.inf)
    for k in range(3):
        sk = s_hat[k]
        if sk == 0.0:
            continue
        bound = vol.box_max[k] if sk > 0.0 else vol.box_min[k]
        tx = np.minimum(tx, (bound - p[:, k]) / sk)
    dl = tx / light_steps
    acc = np.zeros(n)
    for k in range(light_steps):
        q = p + ((k + 0.5) * dl)[:, None] * s_hat[None, :]
        acc += density(vol, q)
    return np.exp(-alpha * dl * acc)


# ---------------------------------------------------------------------------
# The march (Sections 1 and 3)
# ---------------------------------------------------------------------------

DEPTH_ALPHA_MIN = 0.01


def march_rays(vol: OracleVolume, origins, dirs, params, jitter=None,
               return_lookups: bool = False, return_trace: bool = False,
               return_depth: bool = False):
    """March n rays; returns RGBA [n,4] (premultiplied colour, alpha = 1 - T).

    origins, dirs: [n,3] (dirs need not be unit length; they are normalised).
    jitter: per-ray offsets j in [0,1), or None for j = 0.5 (R6).
    params: steps, light_steps, alpha, g, sun_dir, sun_color, ambient,
            integration (0 naive, 1 analytic), t_eps.
    return_lookups adds the number of density lookups performed; return_trace
    adds, per ray, the primary samples taken and a mask with bit i set when
    sample i ran the light march; return_depth adds each ray's representative
    depth (reading R18): the mean sample distance t_i weighted by the opacity
    each step adds, T_before - T_after, when alpha >= DEPTH_ALPHA_MIN; the
    middle of the ray's chord through the box below that; 0 (at infinity)
    for rays that miss the box.
    Each primary step (Section 1): sample rho, march towards the sun for the
    incident light, add the ambient term, integrate over the step (Section
    3.1), update T, stop once T < t_eps (R12)."""
    o = np.asarray(origins, dtype=np.float64).reshape(-1, 3)
    d = _normalize(np.asarray(dirs, dtype=np.float64).reshape(-1, 3))
    n = o.shape[0]
    N, L = int(params.steps), int(params.light_steps)
    alpha = float(params.alpha)
    s_hat = _normalize(np.asarray(params.sun_dir, dtype=np.float64))
    c_sun = np.asarray(params.sun_color, dtype=np.float64)
    c_amb = np.asarray(params.ambient, dtype=np.float64)
    j = np.full(n, 0.5) if jitter is None else np.asarray(jitter, dtype=np.float64)

    tn, tf, hit = ray_box(o, d, vol.box_min, vol.box_max)
    D = np.where(hit, (tf - tn) / N, 0.0)
    phase = hg_phase(d @ s_hat, float(params.g))          # once per pixel (R8)

    T = np.ones(n)
    S = np.zeros((n, 3))
    alive = hit.copy()
    lookups = 0
    prim = np.zeros(n, dtype=np.int64)
    mask = np.zeros(n, dtype=np.uint64)
    opacity_t = np.zeros(n)
    for i in range(N):
        idx = np.nonzero(alive)[0]
        if idx.size == 0:
            break
        t = tn[idx] + (i + j[idx]) * D[idx]
        p = o[idx] + t[:, None] * d[idx]
        rho = density(vol, p)
        lookups += idx.size
        prim[idx] += 1
        TL = np.ones(idx.size)
        lit = rho > 0.0
        if L > 0 and lit.any():
            TL[lit] = light_transmittance(vol, p[lit], s_hat, L, alpha)
            lookups += L * int(lit.sum())
            if i < 64:
                mask[idx[lit]] |= np.uint64(1) << np.uint64(i)
        L_in = c_sun[None, :] * (phase[idx] * TL)[:, None] + c_amb[None, :]
        x = rho * alpha * D[idx]
        T_before = T[idx].copy()
        if int(params.integration) == 1:
            # Section 3.1: S += T0 * L_in * (1 - e^{-x}) (R1, R2), then T update.
            S[idx] += (T[idx] * -np.expm1(-x))[:, None] * L_in
            T[idx] = T[idx] * np.exp(-x)
        else:
            # Section 3.1, basic approach: update T first, then use it (R3).
            T[idx] = T[idx] * np.exp(-x)
            S[idx] += (T[idx] * x)[:, None] * L_in
        opacity_t[idx] += (T_before - T[idx]) * t
        eps = float(params.t_eps)
        if eps > 0.0:
            alive[idx] = T[idx] >= eps
    rgba = np.concatenate([S, (1.0 - T)[:, None]], axis=1)
    rgba[~hit] = 0.0
    extra = ([lookups] if return_lookups else []) + ([(prim, mask)] if return_trace else [])
    if return_depth:
        a = 1.0 - T
        with np.errstate(divide="ignore", invalid="ignore"):
            depth = np.where(a >= DEPTH_ALPHA_MIN, opacity_t / a, 0.5 * (tn + tf))
        extra.append(np.where(hit, depth, 0.0))
    return (rgba, *extra) if extra else rgba


def render(vol: OracleVolume, cam, params, width: int, height: int, frame: int = 0,
           pixels=None, return_lookups: bool = False, return_trace: bool = False,
           return_depth: bool = False):
    """Render the cloud layer (RGBA premultiplied, no background; R15).

    pixels: None for the whole image ([height, width, 4] result), or an
    [n,2] array of (px, py) for those pixels only ([n,4] result).
    return_lookups / return_trace / return_depth: as in march_rays (per-pixel
    results in the result's pixel order; the depth as [height, width] for a
    whole image)."""
    if pixels is None:
        py, px = np.meshgrid(np.arange(height), np.arange(width), indexing="ij")
        px, py = px.reshape(-1), py.reshape(-1)
    else:
        pixels = np.asarray(pixels, dtype=np.int64).reshape(-1, 2)
        px, py = pixels[:, 0], pixels[:, 1]
    o, d = camera_rays(cam, width, height, px, py)
    j = jitter_for(int(params.jitter), px, py, frame, int(params.seed))
    out = march_rays(vol, o, d, params, jitter=j, return_lookups=return_lookups,
                     return_trace=return_trace, return_depth=return_depth)
    if not (return_lookups or return_trace or return_depth):
        out = (out,)
    out = list(out)
    if pixels is None:
        out[0] = out[0].reshape(height, width, 4)
        if return_depth:
            out[-1] = out[-1].reshape(height, width)
    return tuple(out) if len(out) > 1 else out[0]


# ---------------------------------------------------------------------------
# Scalar march in plain Python floats (brute force for tiny cases)
# ---------------------------------------------------------------------------

def _scalar_trilinear(vol, f, repeat):
    nz, ny, nx = vol.shape
    ks, ws = [], []
    for fk, n in zip(f, (nx, ny, nz)):
        k0 = math.floor(fk)
        w = fk - k0
        k1 = k0 + 1
        if repeat:
            k0, k1 = k0 % n, k1 % n
        else:
            k0, k1 = min(max(k0, 0), n - 1), min(max(k1, 0), n - 1)
        ks.append((k0, k1))
        ws.append(w)
    (x0, x1), (y0, y1), (z0, z1) = ks
    wx, wy, wz = ws
    v = vol

    def lerp(a, b, w):
        return a + w * (b - a)

    c00 = lerp(float(v[z0, y0, x0]), float(v[z0, y0, x1]), wx)
    c10 = lerp(float(v[z0, y1, x0]), float(v[z0, y1, x1]), wx)
    c01 = lerp(float(v[z1, y0, x0]), float(v[z1, y0, x1]), wx)
    c11 = lerp(float(v[z1, y1, x0]), float(v[z1, y1, x1]), wx)
    return lerp(lerp(c00, c10, wy), lerp(c01, c11, wy), wz)


def _scalar_density(vol: OracleVolume, p):
    uvw = [(p[k] - vol.box_min[k]) / (vol.box_max[k] - vol.box_min[k]) for k in range(3)]
    nz, ny, nx = vol.base.shape
    b = _scalar_trilinear(vol.base, [uvw[0] * nx - 0.5, uvw[1] * ny - 0.5, uvw[2] * nz - 0.5], False)
    if vol.detail is None:
        return b
    dz, dy, dx = vol.detail.shape
    t = vol.detail_tiling
    d = _scalar_trilinear(vol.detail, [uvw[0] * t * dx - 0.5, uvw[1] * t * dy - 0.5,
                                       uvw[2] * t * dz - 0.5], True)
    we = vol.detail_weight
    return min(max((b - we * d) / (1.0 - we * d), 0.0), 1.0)


def march_ray(vol: OracleVolume, o, d, params, j: float = 0.5):
    """One ray, plain Python floats: an independent restatement of march_rays
    used as a brute-force check on tiny inputs. Returns (r, g, b, a)."""
    o = [float(c) for c in o]
    nd = math.sqrt(sum(float(c) ** 2 for c in d))
    d = [float(c) / nd for c in d]
    tn, tf = 0.0, math.inf
    for k in range(3):
        if d[k] == 0.0:
            if not (vol.box_min[k] <= o[k] <= vol.box_max[k]):
                return (0.0, 0.0, 0.0, 0.0)
            continue
        t0 = (vol.box_min[k] - o[k]) / d[k]
        t1 = (vol.box_max[k] - o[k]) / d[k]
        tn = max(tn, min(t0, t1))
        tf = min(tf, max(t0, t1))
    if not tf > tn:
        return (0.0, 0.0, 0.0, 0.0)
    N, L = int(params.steps), int(params.light_steps)
    D = (tf - tn) / N
    ns = math.sqrt(sum(float(c) ** 2 for c in params.sun_dir))
    s = [float(c) / ns for c in params.sun_dir]
    g = float(params.g)
    mu = sum(d[k] * s[k] for k in range(3))
    phase = (1.0 - g * g) / (4.0 * math.pi * (1.0 + g * g - 2.0 * g * mu) ** 1.5)
    alpha = float(params.alpha)
    T, S = 1.0, [0.0, 0.0, 0.0]
    for i in range(N):
        t = tn + (i + j) * D
        p = [o[k] + t * d[k] for k in range(3)]
        rho = _scalar_density(vol, p)
        TL = 1.0
        if rho > 0.0 and L > 0:
            tx = math.inf
            for k in range(3):
                if s[k] != 0.0:
                    bound = vol.box_max[k] if s[k] > 0.0 else vol.box_min[k]
                    tx = min(tx, (bound - p[k]) / s[k])
            dl = tx / L
            acc = 0.0
            for k in range(L):
                acc += _scalar_density(vol, [p[c] + (k + 0.5) * dl * s[c] for c in range(3)])
            TL = math.exp(-alpha * dl * acc)
        L_in = [params.sun_color[c] * phase * TL + params.ambient[c] for c in range(3)]
        x = rho * alpha * D
        if int(params.integration) == 1:
            f = T * -math.expm1(-x)
            S = [S[c] + f * L_in[c] for c in range(3)]
            T = T * math.exp(-x)
        else:
            T = T * math.exp(-x)
            S = [S[c] + T * x * L_in[c] for c in range(3)]
        if params.t_eps > 0.0 and T < params.t_eps:
            break
    return (S[0], S[1], S[2], 1.0 - T)


# ---------------------------------------------------------------------------
# Temporal resolve (Section 3.2; reading R13)
# ---------------------------------------------------------------------------

def taa_resolve(cur, hist, blend: float, frame_index: int):
    """Accumulate the jittered frames: clamp the history into the 3x3
    neighbourhood min/max of the current frame (edge-clamped), then blend
    out = h + blend * (cur - h). Frame 0, or no history, copies cur."""
    cur = np.asarray(cur, dtype=np.float64)
    if hist is None or int(frame_index) == 0:
        return cur.copy()
    hist = np.asarray(hist, dtype=np.float64)
    H, W = cur.shape[:2]
    pad = np.pad(cur, ((1, 1), (1, 1), (0, 0)), mode="edge")
    nb = np.stack([pad[dy:dy + H, dx:dx + W] for dy in range(3) for dx in range(3)])
    lo, hi = nb.min(axis=0), nb.max(axis=0)
    h = np.minimum(np.maximum(hist, lo), hi)
    return h + blend * (cur - h)


def camera_project(cam, width: int, height: int, v):
    """Continuous pixel coordinates (u, w) of directions v [n,3] (camera-space
    vectors from the camera's position) for the pinhole of camera_rays: pixel
    (px, py)'s centre direction maps to (px, py). Also returns z = v . forward
    (the point is behind the camera when z <= 0)."""
    pos = np.asarray(cam.pos, dtype=np.float64)
    f = _normalize(np.asarray(cam.target, dtype=np.float64) - pos)
    r = _normalize(np.cross(f, np.asarray(cam.up, dtype=np.float64)))
    u = np.cross(r, f)
    tan_half = math.tan(math.radians(cam.vfov_deg) * 0.5)
    z = v @ f
    with np.errstate(divide="ignore", invalid="ignore"):
        x = (v @ r) / z
        y = (v @ u) / z
    uc = (x / (tan_half * (width / height)) + 1.0) * (width * 0.5) - 0.5
    wc = (1.0 - y / tan_half) * (height * 0.5) - 0.5
    return uc, wc, z


def taa_resolve_reproject(cur, hist, depth, cam, prev_cam, blend: float, frame_index: int):
    """Temporal resolve with camera reprojection (Section 3.2 names Playdead's
    TAA, whose history is reprojected; reading R18). For each pixel, the point
    at its representative depth along its ray (at infinity for depth 0) is
    projected into the previous camera; the history is sampled there
    bilinearly with edge clamping, then clamped into the current 3x3
    neighbourhood min/max and blended, out = h + blend * (cur - h). A point
    behind the previous camera or outside its image uses the current value
    as history. Frame 0, or no history, copies cur."""
    cur = np.asarray(cur, dtype=np.float64)
    if hist is None or int(frame_index) == 0:
        return cur.copy()
    hist = np.asarray(hist, dtype=np.float64)
    H, W = cur.shape[:2]
    py, px = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    o, d = camera_rays(cam, W, H, px.reshape(-1), py.reshape(-1))
    dep = np.asarray(depth, dtype=np.float64).reshape(-1)
    prev_pos = np.asarray(prev_cam.pos, dtype=np.float64)
    v = np.where((dep > 0.0)[:, None], o + dep[:, None] * d - prev_pos[None, :], d)
    uc, wc, z = camera_project(prev_cam, W, H, v)
    valid = (z > 0.0) & (uc >= -0.5) & (uc <= W - 0.5) & (wc >= -0.5) & (wc <= H - 0.5)
    uc = np.where(valid, uc, 0.0)
    wc = np.where(valid, wc, 0.0)
    x0f, y0f = np.floor(uc), np.floor(wc)
    fx, fy = (uc - x0f)[:, None], (wc - y0f)[:, None]
    x0 = np.clip(x0f.astype(np.int64), 0, W - 1)
    x1 = np.clip(x0f.astype(np.int64) + 1, 0, W - 1)
    y0 = np.clip(y0f.astype(np.int64), 0, H - 1)
    y1 = np.clip(y0f.astype(np.int64) + 1, 0, H - 1)
    top = _lerp(hist[y0, x0], hist[y0, x1], fx)
    bot = _lerp(hist[y1, x0], hist[y1, x1], fx)
    h = _lerp(top, bot, fy)
    c = cur.reshape(-1, 4)
    h = np.where(valid[:, None], h, c)
    pad = np.pad(cur, ((1, 1), (1, 1), (0, 0)), mode="edge")
    nb = np.stack([pad[dy:dy + H, dx:dx + W] for dy in range(3) for dx in range(3)])
    lo, hi = nb.min(axis=0).reshape(-1, 4), nb.max(axis=0).reshape(-1, 4)
    h = np.minimum(np.maximum(h, lo), hi)
    return (h + blend * (c - h)).reshape(H, W, 4)


# ---------------------------------------------------------------------------
# Composite of the resolved low-resolution cloud layer into the scene
# (Section 3.2; reading R19)
# ---------------------------------------------------------------------------

def upsample_bilinear(img, width: int, height: int):
    """Bilinear resize of img [h][w][c] to [height][width][c] with pixel
    centres aligned: output pixel x samples the input at (x + 1/2) w / width
    - 1/2 (likewise in y), edge-clamped."""
    img = np.asarray(img, dtype=np.float64)
    h, w = img.shape[:2]
    uc = (np.arange(width) + 0.5) * (w / width) - 0.5
    vc = (np.arange(height) + 0.5) * (h / height) - 0.5
    x0f, y0f = np.floor(uc), np.floor(vc)
    fx, fy = (uc - x0f)[None, :, None], (vc - y0f)[:, None, None]
    x0 = np.clip(x0f.astype(np.int64), 0, w - 1)
    x1 = np.clip(x0f.astype(np.int64) + 1, 0, w - 1)
    y0 = np.clip(y0f.astype(np.int64), 0, h - 1)
    y1 = np.clip(y0f.astype(np.int64) + 1, 0, h - 1)
    top = _lerp(img[y0][:, x0], img[y0][:, x1], fx)
    bot = _lerp(img[y1][:, x0], img[y1][:, x1], fx)
    return _lerp(top, bot, fy)


def composite(cloud, background):
    """Premultiplied cloud layer (any resolution) over the background
    [height][width][4]: the layer is up-sampled bilinearly to the background's
    size, then out = c + (1 - c_alpha) * bg in every channel."""
    bg = np.asarray(background, dtype=np.float64)
    H, W = bg.shape[:2]
    c = upsample_bilinear(cloud, W, H)
    return c + (1.0 - c[..., 3:4]) * bg

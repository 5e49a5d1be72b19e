"""Seeded synthetic inputs: density volumes, cameras and render settings.

This module produces the *inputs* of a cloud render and nothing else. It holds
none of the method's arithmetic (no ray generation, marching, lighting,
integration, jitter hash or temporal filter); both the HIP library and the CPU
oracle consume what it returns.

The paper (Section 4) renders its own game scene, which is not published, so
every workload here is a seeded procedural cloud volume of the kind the paper
describes in Section 1 (a 3-D density field sampled along rays) and that its
cited prior work builds from noise (Schneider and Vos 2015):

* value-noise fractal Brownian motion (FBM), tileable, with a quintic fade,
  remapped by a coverage threshold to [0, 1];
* an optional height profile that confines the clouds to a slab layer;
* a tileable detail volume (Worley F1 plus value noise) for erosion.

Volumes are laid out ``[nz][ny][nx]`` with x fastest and y the height axis, over
the world box ``[-0.5, 0.5]^3``. Lattice values come from numpy's PCG64
generator seeded by ``(seed, octave)``; nothing here draws from the jitter hash
the renderer uses.
"""

from __future__ import annotations

import hashlib
import math
import os
from dataclasses import dataclass, field, replace
from typing import Optional, Sequence

import numpy as np

BOX_MIN = (-0.5, -0.5, -0.5)
BOX_MAX = (0.5, 0.5, 0.5)

# Light set-up shared by every workload: sun direction (towards the sun),
# sun colour times intensity, and the ambient colour (Section 1 names the
# terms; the values are this project's choice).
SUN_DIR = (0.3, 0.8, 0.5)
SUN_COLOR = (4.0, 3.8, 3.6)
AMBIENT = (0.2, 0.2, 0.2)
JITTER_SEED = 1609


# ----------------------------------------------------------------------------
# Noise volumes
# ----------------------------------------------------------------------------

def _fade(t: np.ndarray) -> np.ndarray:
    """Quintic smoothstep 6t^5 - 15t^4 + 10t^3 (C2-continuous value noise)."""
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def _axis_weights(n: int, freq: int) -> np.ndarray:
    """Dense [n, freq] matrix that interpolates a periodic lattice of ``freq``
    cells onto ``n`` texel centres along one axis (two non-zeros per row)."""
    u = (np.arange(n, dtype=np.float64) + 0.5) / n * freq
    i0 = np.floor(u).astype(np.int64)
    w = _fade(u - i0)
    m = np.zeros((n, freq), dtype=np.float64)
    rows = np.arange(n)
    np.add.at(m, (rows, i0 % freq), 1.0 - w)
    np.add.at(m, (rows, (i0 + 1) % freq), w)
    return m


def _lattice(seed: int, octave: int, shape) -> np.ndarray:
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), int(octave), 0x5C3]))
    return rng.random(shape)


def value_noise(n: int, freq: int, seed: int, octave: int) -> np.ndarray:
    """One tileable value-noise octave sampled at the centres of an n^3 grid."""
    lat = _lattice(seed, octave, (freq, freq, freq))  # [c=z][b=y][a=x]
    m = _axis_weights(n, freq)
    a = np.tensordot(lat, m, axes=([2], [1]))          # [c][b][x]
    b = np.tensordot(m, a, axes=([1], [1]))            # [y][c][x]
    b = np.ascontiguousarray(b.transpose(1, 0, 2))     # [c][y][x]
    return np.tensordot(m, b, axes=([1], [0]))         # [z][y][x]


def value_fbm(n: int, octaves: int, seed: int, base_freq: int = 4,
              lacunarity: int = 2, gain: float = 0.5) -> np.ndarray:
    """Tileable FBM in [0, 1], normalised by the sum of octave amplitudes."""
    out = np.zeros((n, n, n), dtype=np.float64)
    amp, total = 1.0, 0.0
    for o in range(octaves):
        out += amp * value_noise(n, base_freq * lacunarity ** o, seed, o)
        total += amp
        amp *= gain
    return out / total


def coverage_remap(noise: np.ndarray, coverage: float) -> np.ndarray:
    """Keep only noise above the coverage threshold, rescaled to [0, 1]."""
    return np.clip((noise - coverage) / (1.0 - coverage), 0.0, 1.0)


def _smoothstep(e0: float, e1: float, x: np.ndarray) -> np.ndarray:
    t = np.clip((x - e0) / (e1 - e0), 0.0, 1.0)
    return t * t * (3.0 - 2.0 * t)


def height_profile(n: int) -> np.ndarray:
    """Slab layer: zero below 15 % and above 85 % of the box height."""
    v = (np.arange(n, dtype=np.float64) + 0.5) / n
    return _smoothstep(0.15, 0.30, v) * (1.0 - _smoothstep(0.55, 0.85, v))


def worley_f1(n: int, freq: int, seed: int, octave: int) -> np.ndarray:
    """Tileable Worley F1 (distance to nearest feature point, in cell units)
    with one feature point per cell, on an n^3 grid of texel centres."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), int(octave), 0x3017]))
    pts = rng.random((freq, freq, freq, 3))  # offset within cell, (x, y, z)
    c = (np.arange(n, dtype=np.float64) + 0.5) / n * freq
    gz, gy, gx = np.meshgrid(c, c, c, indexing="ij")
    cz, cy, cx = (np.floor(g).astype(np.int64) for g in (gz, gy, gx))
    best = np.full(gz.shape, np.inf)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                kz, ky, kx = cz + dz, cy + dy, cx + dx
                off = pts[kz % freq, ky % freq, kx % freq]
                d2 = ((kx + off[..., 0] - gx) ** 2 + (ky + off[..., 1] - gy) ** 2
                      + (kz + off[..., 2] - gz) ** 2)
                best = np.minimum(best, d2)
    return np.sqrt(best)


def detail_noise(n: int, seed: int) -> np.ndarray:
    """Tileable detail in [0, 1]: half 3-octave inverted Worley (frequencies
    4, 8, 16), half 3-octave value FBM."""
    acc, tot = 0.0, 0.0
    for o, f in enumerate((4, 8, 16)):
        w = 1.0 - np.minimum(worley_f1(n, f, seed, o), 1.0)
        acc = acc + 0.5 ** o * w
        tot += 0.5 ** o
    return 0.5 * (acc / tot) + 0.5 * value_fbm(n, 3, seed + 1000, base_freq=4)


@dataclass(frozen=True)
class VolumeSpec:
    n: int
    octaves: int
    coverage: float
    seed: int
    height_falloff: bool = False

    def key(self) -> str:
        s = f"v1|{self.n}|{self.octaves}|{self.coverage}|{self.seed}|{self.height_falloff}"
        return hashlib.sha1(s.encode()).hexdigest()[:16]


def _cache_dir() -> Optional[str]:
    d = os.environ.get("CLOUD_VOLUME_CACHE",
                       os.path.join(os.environ.get("TMPDIR", "/tmp"), "cloud_volumes"))
    try:
        os.makedirs(d, exist_ok=True)
        return d
    except OSError:
        return None


def make_density(spec: VolumeSpec, cache: bool = True) -> np.ndarray:
    """Seeded FP64 density volume [n][n][n] in [0, 1] (cached on disk)."""
    d = _cache_dir() if cache else None
    path = os.path.join(d, f"density_{spec.key()}.npy") if d else None
    if path and os.path.exists(path):
        return np.load(path)
    rho = coverage_remap(value_fbm(spec.n, spec.octaves, spec.seed), spec.coverage)
    if spec.height_falloff:
        rho = rho * height_profile(spec.n)[None, :, None]
    if path:
        tmp = f"{path}.{os.getpid()}.tmp.npy"
        np.save(tmp, rho)
        os.replace(tmp, path)
    return rho


def make_detail(n: int, seed: int, cache: bool = True) -> np.ndarray:
    d = _cache_dir() if cache else None
    path = os.path.join(d, f"detail_{n}_{seed}.npy") if d else None
    if path and os.path.exists(path):
        return np.load(path)
    det = detail_noise(n, seed)
    if path:
        tmp = f"{path}.{os.getpid()}.tmp.npy"
        np.save(tmp, det)
        os.replace(tmp, path)
    return det


def quantise(x: np.ndarray, dtype: str) -> np.ndarray:
    """Round an FP64 volume to its storage type (round to nearest even).

    Returns the stored array: float32, float16, or for bf16 a uint16 array of
    bfloat16 bit patterns."""
    if dtype == "f32":
        return x.astype(np.float32)
    if dtype == "f16":
        return x.astype(np.float16)
    if dtype == "bf16":
        f = x.astype(np.float32).view(np.uint32).astype(np.uint64)
        rounded = (f + 0x7FFF + ((f >> 16) & 1)) >> 16
        return rounded.astype(np.uint16)
    raise ValueError(dtype)


def decode(stored: np.ndarray, dtype: str) -> np.ndarray:
    """Exact FP64 values of a stored volume."""
    if dtype in ("f32", "f16"):
        return stored.astype(np.float64)
    if dtype == "bf16":
        return (stored.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    raise ValueError(dtype)


# ----------------------------------------------------------------------------
# Cameras and render settings
# ----------------------------------------------------------------------------

@dataclass(frozen=True)
class Camera:
    pos: tuple
    target: tuple = (0.0, 0.0, 0.0)
    up: tuple = (0.0, 1.0, 0.0)
    vfov_deg: float = 60.0


def orbit_camera(radius: float, azimuth_deg: float, elevation_deg: float,
                 vfov_deg: float = 60.0) -> Camera:
    """Camera on a sphere around the box centre, looking at the centre."""
    ph, th = math.radians(azimuth_deg), math.radians(elevation_deg)
    pos = (radius * math.sin(ph) * math.cos(th), radius * math.sin(th),
           radius * math.cos(ph) * math.cos(th))
    return Camera(pos=pos, vfov_deg=vfov_deg)


@dataclass(frozen=True)
class Params:
    """Render settings (names follow the paper: alpha is the extinction per
    unit density, g the Henyey-Greenstein asymmetry)."""
    steps: int = 8
    light_steps: int = 6
    alpha: float = 10.0
    g: float = 0.6
    sun_dir: tuple = SUN_DIR
    sun_color: tuple = SUN_COLOR
    ambient: tuple = AMBIENT
    jitter: int = 1             # 0: fixed 0.5; 1: per pixel; 2: per 8x8 tile; 3: per frame
    seed: int = JITTER_SEED
    integration: int = 1        # 0: naive S = T L; 1: analytic
    t_eps: float = 1e-5         # early-out threshold on transmittance (0 = off)
    detail_weight: float = 0.3
    detail_tiling: float = 4.0


@dataclass(frozen=True)
class Workload:
    name: str
    width: int
    height: int
    volume: VolumeSpec
    dtype: str
    params: Params
    radius: float
    elevation_deg: float
    azimuth0_deg: float = 210.0
    frames: int = 1
    taa_blend: float = 0.1
    detail_n: int = 0           # 0: no detail volume
    detail_seed: int = 33
    views: int = 1
    description: str = ""
    display: tuple = ()         # (width, height) the cloud layer is composited at; () = none

    def camera(self, frame: int = 0, view: int = 0) -> Camera:
        """Orbit advancing 1 degree per frame; views spread 45 degrees apart."""
        return orbit_camera(self.radius, self.azimuth0_deg + frame + 45.0 * view,
                            self.elevation_deg)


WORKLOADS = {
    "C1": Workload(
        "C1", 64, 64, VolumeSpec(32, 3, 0.5, seed=1), "f32",
        Params(steps=128, light_steps=6, alpha=8.0, g=0.6, jitter=0),
        radius=2.0, elevation_deg=20.0,
        description="tiny: 64x64, 32^3 f32, 128 unjittered steps"),
    "C2": Workload(
        "C2", 1280, 720, VolumeSpec(256, 5, 0.45, seed=2, height_falloff=True), "f32",
        Params(steps=8, alpha=10.0, g=0.6, jitter=1),
        radius=1.0, elevation_deg=10.0, frames=16,
        description="720p, 256^3 f32 slab layer, 8 jittered steps + TAA, 16-frame orbit"),
    "C2ref": Workload(
        "C2ref", 1280, 720, VolumeSpec(256, 5, 0.45, seed=2, height_falloff=True), "f32",
        Params(steps=128, alpha=10.0, g=0.6, jitter=0),
        radius=1.0, elevation_deg=10.0, frames=16,
        description="C2's 128-step unjittered reference"),
    "C3": Workload(
        "C3", 1920, 1080, VolumeSpec(128, 5, 0.45, seed=3), "f16",
        Params(steps=16, alpha=10.0, g=0.7, jitter=1),
        radius=1.0, elevation_deg=10.0, detail_n=32, detail_seed=33,
        description="1080p, 128^3 f16 base + 32^3 f16 detail (erosion 0.3), 16 jittered steps"),
    "H": Workload(
        "H", 1920, 1080, VolumeSpec(256, 5, 0.45, seed=2, height_falloff=True), "f32",
        Params(steps=8, alpha=10.0, g=0.6, jitter=1),
        radius=1.0, elevation_deg=10.0, frames=16,
        description="1080p, 256^3 f32 slab layer, 8 jittered steps, 6 light steps, TAA"),
    "Hh": Workload(
        "Hh", 960, 540, VolumeSpec(256, 5, 0.45, seed=2, height_falloff=True), "f32",
        Params(steps=8, alpha=10.0, g=0.6, jitter=1),
        radius=1.0, elevation_deg=10.0, frames=16, display=(1920, 1080),
        description="half-resolution cloud layer (960x540) of H, resolved, up-sampled and "
                    "composited over a 1920x1080 sky"),
    "Hq": Workload(
        "Hq", 480, 270, VolumeSpec(256, 5, 0.45, seed=2, height_falloff=True), "f32",
        Params(steps=8, alpha=10.0, g=0.6, jitter=1),
        radius=1.0, elevation_deg=10.0, frames=16, display=(1920, 1080),
        description="quarter-resolution cloud layer (480x270) of H, resolved, up-sampled and "
                    "composited over a 1920x1080 sky"),
    "C5": Workload(
        "C5", 3840, 2160, VolumeSpec(512, 6, 0.5, seed=5), "f16",
        Params(steps=8, alpha=10.0, g=0.6, jitter=1),
        radius=1.0, elevation_deg=10.0, frames=16, views=8,
        description="4K x 8 views, 512^3 f16, 8 jittered steps + TAA"),
}


def workload(name: str, **overrides) -> Workload:
    w = WORKLOADS[name]
    if overrides:
        pov = {k: v for k, v in overrides.items() if k in Params.__dataclass_fields__}
        wov = {k: v for k, v in overrides.items() if k not in pov}
        if pov:
            wov["params"] = replace(w.params, **pov)
        w = replace(w, **wov)
    return w


def sky_background(width: int, height: int) -> np.ndarray:
    """A [height][width][4] float32 sky (opaque, alpha 1) to composite the cloud
    layer over: a vertical blend from a pale horizon (bottom row) to a deeper
    zenith colour (top row), with a faint horizontal tint so that rows are
    not constant. Input data only."""
    v = 1.0 - (np.arange(height, dtype=np.float64) + 0.5) / height      # 1 at the top
    u = (np.arange(width, dtype=np.float64) + 0.5) / width
    horizon = np.array([0.80, 0.85, 0.95])
    zenith = np.array([0.20, 0.40, 0.85])
    w = np.sqrt(v)[:, None, None]
    rgb = horizon[None, None, :] * (1.0 - w) + zenith[None, None, :] * w
    rgb = rgb * (0.95 + 0.05 * u)[None, :, None]
    out = np.concatenate([rgb, np.ones((height, width, 1))], axis=-1)
    return out.astype(np.float32)


@dataclass
class Scene:
    """Stored volumes of a workload plus their exact FP64 decodings."""
    workload: Workload
    base_stored: np.ndarray
    base_f64: np.ndarray
    detail_stored: Optional[np.ndarray] = None
    detail_f64: Optional[np.ndarray] = None


def make_scene(w: Workload, dtype: Optional[str] = None, cache: bool = True) -> Scene:
    dt = dtype or w.dtype
    base = quantise(make_density(w.volume, cache=cache), dt)
    det_s = det_f = None
    if w.detail_n:
        det_s = quantise(make_detail(w.detail_n, w.detail_seed, cache=cache), dt)
        det_f = decode(det_s, dt)
    return Scene(w, base, decode(base, dt), det_s, det_f)


def random_pixels(width: int, height: int, count: int, seed: int) -> np.ndarray:
    """Seeded sample of distinct pixel coordinates, [count][2] as (px, py)."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), width, height]))
    count = min(count, width * height)
    idx = rng.choice(width * height, size=count, replace=False)
    return np.stack([idx % width, idx // width], axis=1).astype(np.int64)

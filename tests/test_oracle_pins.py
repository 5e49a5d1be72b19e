"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test states the closed form, invariant or brute-force check it uses and
the passage it follows. They are chosen so that a plausible slip anywhere in
the oracle (a dropped term, a wrong sign or index, a swapped operand) fails at
least one of them.
"""

import math
import os
from dataclasses import replace

import numpy as np
import pytest

from oracle import cloud as O
from paper_1609_05344_amd import scenes

HERE = os.path.dirname(os.path.abspath(__file__))


def params(**kw):
    base = scenes.Params(steps=8, light_steps=6, alpha=10.0, g=0.6, jitter=0, t_eps=0.0)
    return replace(base, **kw)


def const_volume(c, n=8, **kw):
    return O.OracleVolume(base=np.full((n, n, n), float(c)), **kw)


def one_ray(vol, o, d, p, j=None):
    jj = None if j is None else np.array([j], dtype=np.float64)
    return O.march_rays(vol, np.array([o], float), np.array([d], float), p, jitter=jj)[0]


# ---------------------------------------------------------------------------
# Pi1: Henyey-Greenstein phase (Section 1) -- normalisation by quadrature
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("g,npts", [(-0.5, 64), (0.0, 64), (0.3, 64), (0.6, 64), (0.7, 64), (0.9, 512)])
def test_hg_normalised_and_mean_cosine(g, npts):
    x, w = np.polynomial.legendre.leggauss(npts)
    p = O.hg_phase(x, g)
    assert abs(2 * math.pi * np.sum(w * p) - 1.0) < 1e-12
    assert abs(2 * math.pi * np.sum(w * x * p) - g) < 1e-12


def test_hg_spot_values():
    # (1-g^2)/(4 pi (1 -+ g)^3): forward and backward peaks.
    assert O.hg_phase(1.0, 0.6) == pytest.approx(0.795775, abs=1e-6)
    assert O.hg_phase(-1.0, 0.6) == pytest.approx(0.012434, abs=1e-6)
    assert O.hg_phase(1.0, 0.7) == pytest.approx(1.503130, abs=1e-6)
    assert O.hg_phase(-1.0, 0.7) == pytest.approx(0.008261, abs=1e-6)
    assert O.hg_phase(0.3, 0.0) == pytest.approx(1 / (4 * math.pi), abs=1e-15)


# ---------------------------------------------------------------------------
# Rays and the box (Section 1: one ray per pixel, marched to where it leaves the volume)
# ---------------------------------------------------------------------------

def test_camera_single_pixel_looks_at_target():
    cam = scenes.orbit_camera(2.0, 210.0, 20.0)
    o, d = O.camera_rays(cam, 1, 1, np.array([0]), np.array([0]))
    f = -np.asarray(cam.pos) / np.linalg.norm(cam.pos)
    assert np.allclose(d[0], f, atol=1e-15)
    assert np.allclose(o[0], cam.pos, atol=0)


@pytest.mark.parametrize("W,H", [(65, 33), (1921, 1081)])
def test_camera_field_of_view(W, H):
    cam = scenes.Camera(pos=(0.0, 0.0, 3.0), vfov_deg=60.0)
    tan_half = math.tan(math.radians(30.0))
    # top row, centre column: row 0 is at the top (+up), vertical FOV
    _, d = O.camera_rays(cam, W, H, np.array([(W - 1) // 2]), np.array([0]))
    assert d[0, 1] > 0
    assert d[0, 1] / -d[0, 2] == pytest.approx((1 - 1 / H) * tan_half, rel=1e-13)
    # right column, centre row: horizontal extent scaled by the aspect ratio
    _, d = O.camera_rays(cam, W, H, np.array([W - 1]), np.array([(H - 1) // 2]))
    # camera looks down -z with up +y, so right is +x
    assert d[0, 0] / -d[0, 2] == pytest.approx((1 - 1 / W) * tan_half * W / H, rel=1e-13)


def test_ray_box_cases():
    bmin, bmax = (-0.5,) * 3, (0.5,) * 3
    o = np.array([[0, 2, 0], [0, 0, 0], [0.7, 2, 0], [0.5, 2, 0], [3, 3, 3], [0, 2, 0]], float)
    d = np.array([[0, -1, 0], [1, 0, 0], [0, -1, 0], [0, -1, 0], [-1, -1, -1], [0, 1, 0]], float)
    d[4] /= np.sqrt(3)
    tn, tf, hit = O.ray_box(o, d, bmin, bmax)
    assert hit.tolist() == [True, True, False, True, True, False]
    assert (tn[0], tf[0]) == (1.5, 2.5)
    assert (tn[1], tf[1]) == (0.0, 0.5)                 # starts inside: t_near = 0
    assert (tn[3], tf[3]) == (1.5, 2.5)                 # on the face plane: inside
    assert tn[4] == pytest.approx(2.5 * math.sqrt(3), rel=1e-15)
    assert tf[4] == pytest.approx(3.5 * math.sqrt(3), rel=1e-15)


# ---------------------------------------------------------------------------
# Pi9: trilinear lookup conventions (reading R10) and erosion (R11)
# ---------------------------------------------------------------------------

def test_trilinear_constant_exact():
    for c in (0.0, 0.3, 1.0, 0.123456789):
        vol = const_volume(c, n=5)
        p = np.random.default_rng(0).uniform(-0.6, 0.6, size=(1000, 3))
        assert np.all(O.density(vol, p) == c)


def test_trilinear_linear_in_x_and_clamp():
    n, a, b = 16, 0.2, 0.5
    xs = a + b * (np.arange(n) + 0.5) / n
    vol = O.OracleVolume(base=np.broadcast_to(xs[None, None, :], (n, n, n)).copy())
    u = np.linspace(0.0, 1.0, 1001)
    p = np.stack([u - 0.5, np.zeros_like(u), np.zeros_like(u)], axis=1)
    rho = O.density(vol, p)
    inner = (u >= 0.5 / n) & (u <= 1 - 0.5 / n)
    assert np.max(np.abs(rho[inner] - (a + b * u[inner]))) < 1e-15
    assert np.all(rho[u < 0.5 / n] == xs[0])
    assert np.all(rho[u > 1 - 0.5 / n] == xs[-1])


def test_trilinear_single_voxel_tent():
    n, k = 8, (3, 5, 2)  # (x, y, z)
    base = np.zeros((n, n, n))
    base[k[2], k[1], k[0]] = 1.0
    vol = O.OracleVolume(base=base)
    p = np.random.default_rng(1).uniform(-0.5, 0.5, size=(4000, 3))
    f = (p + 0.5) * n - 0.5
    tent = np.prod(np.maximum(0.0, 1.0 - np.abs(f - np.array(k))), axis=1)
    assert np.max(np.abs(O.density(vol, p) - tent)) < 1e-14


def test_detail_repeat_and_erosion():
    rng = np.random.default_rng(2)
    det = rng.uniform(0, 1, size=(4, 4, 4))
    vol = O.OracleVolume(base=np.full((6, 6, 6), 0.7), detail=det,
                         detail_weight=0.3, detail_tiling=4.0)
    p = rng.uniform(-0.5, 0.25, size=(500, 3))
    r0 = O.density(vol, p)
    # repeat addressing: a shift by one tile (1/tiling of the box) changes nothing
    r1 = O.density(vol, p + np.array([0.25, 0.0, 0.0]))
    r2 = O.density(vol, p + np.array([0.0, 0.25, 0.25]))
    assert np.max(np.abs(r0 - r1)) < 1e-12 and np.max(np.abs(r0 - r2)) < 1e-12
    # constant detail -> closed form of the erosion
    vol_c = O.OracleVolume(base=np.full((6, 6, 6), 0.7), detail=np.full((4, 4, 4), 0.5),
                           detail_weight=0.3, detail_tiling=4.0)
    assert np.allclose(O.density(vol_c, p), (0.7 - 0.15) / (1 - 0.15), atol=1e-15)
    # cores survive, thin edges vanish
    for b, expect in ((1.0, 1.0), (0.0, 0.0), (0.1, 0.0)):
        v = O.OracleVolume(base=np.full((6, 6, 6), b), detail=np.full((4, 4, 4), 0.9),
                           detail_weight=0.3, detail_tiling=4.0)
        assert np.allclose(O.density(v, p), expect, atol=1e-15)


# ---------------------------------------------------------------------------
# Pi2, Pi3: homogeneous box -- Beer-Lambert and step-count invariance (3.1)
# ---------------------------------------------------------------------------

RAYS = [((0.0, 2.0, 0.0), (0.0, -1.0, 0.0), 1.0),
        ((-3.0, 0.1, 0.2), (1.0, 0.0, 0.0), 1.0),
        ((2.0, 1.5, 1.7), (-0.9, -0.7, -0.8), None)]


def chord(o, d):
    tn, tf, hit = O.ray_box(np.array([o]), np.array([d]) / np.linalg.norm(d), (-0.5,) * 3, (0.5,) * 3)
    assert hit[0]
    return tf[0] - tn[0]


@pytest.mark.parametrize("N", [1, 3, 8, 128])
@pytest.mark.parametrize("j", [0.0, 0.37, 0.5, 1 - 2 ** -24])
def test_homogeneous_transmittance_and_sun_off(N, j):
    c = 0.4
    for o, d, Hc in RAYS:
        H = chord(o, d) if Hc is None else Hc
        for integ in (0, 1):
            p = params(steps=N, alpha=8.0, integration=integ, sun_color=(0.0, 0.0, 0.0),
                       ambient=(0.2, 0.3, 0.5))
            rgba = one_ray(const_volume(c), o, d, p, j)
            A = -math.expm1(-c * 8.0 * H)
            assert abs(rgba[3] - A) < 1e-13           # Beer-Lambert, both rules
            if integ == 1:                            # analytic: independent of N and j
                assert np.max(np.abs(rgba[:3] - np.array([0.2, 0.3, 0.5]) * A)) < 1e-13


# ---------------------------------------------------------------------------
# Pi4: telescoping -- analytic integration, sun off, any density field
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("N", [1, 8, 37, 128])
def test_telescoping_any_volume(N):
    rho = scenes.make_density(scenes.WORKLOADS["C1"].volume, cache=False)
    vol = O.OracleVolume(base=rho)
    cam = scenes.orbit_camera(2.0, 210.0, 20.0)
    pix = scenes.random_pixels(64, 64, 300, seed=7)
    p = params(steps=N, alpha=8.0, sun_color=(0, 0, 0), ambient=(0.2, 0.25, 0.3), jitter=1, t_eps=1e-5)
    rgba = O.render(vol, cam, p, 64, 64, frame=3, pixels=pix)
    a = np.array([0.2, 0.25, 0.3])
    assert np.max(np.abs(rgba[:, :3] - a[None, :] * rgba[:, 3:4])) < 1e-13
    assert np.any(rgba[:, 3] > 0.3)


# ---------------------------------------------------------------------------
# Pi5: the naive rule depends on the step length and converges (Section 3.1)
# ---------------------------------------------------------------------------

def naive_closed_form(a, x, N):
    return a * x * math.exp(-x) * (-math.expm1(-N * x)) / (-math.expm1(-x))


@pytest.mark.parametrize("N,ratio", [(8, 0.58198), (16, 0.77075), (128, 0.96908), (4096, 0.99902)])
def test_naive_step_dependence_and_convergence(N, ratio):
    sigH = 8.0
    c = sigH / 10.0      # alpha 10, chord 1
    p_n = params(steps=N, alpha=10.0, integration=0, sun_color=(0, 0, 0), ambient=(0.2, 0.2, 0.2))
    p_a = replace(p_n, integration=1)
    naive = one_ray(const_volume(c), (0, 2, 0), (0, -1, 0), p_n)
    ana = one_ray(const_volume(c), (0, 2, 0), (0, -1, 0), p_a)
    x = sigH / N
    assert abs(naive[0] - naive_closed_form(0.2, x, N)) < 1e-13
    assert naive[0] / ana[0] == pytest.approx(x / math.expm1(x), rel=1e-12)
    assert naive[0] / ana[0] == pytest.approx(ratio, abs=6e-6)
    if N == 4096:       # relative gap ~ x/2 = 9.8e-4
        assert abs(1 - naive[0] / ana[0]) < 1e-3


def test_naive_converges_to_analytic_on_noise():
    rho = scenes.make_density(scenes.WORKLOADS["C1"].volume, cache=False)
    vol = O.OracleVolume(base=rho)
    cam = scenes.orbit_camera(2.0, 210.0, 20.0)
    pix = scenes.random_pixels(64, 64, 24, seed=11)
    p_a = params(steps=4096, alpha=8.0, integration=1)
    p_n = replace(p_a, integration=0)
    a = O.render(vol, cam, p_a, 64, 64, pixels=pix)
    n = O.render(vol, cam, p_n, 64, 64, pixels=pix)
    # per step |analytic - naive| <= T L x^2 / 2; x <= alpha * max(rho) * chord / N
    xmax = 8.0 * rho.max() * math.sqrt(3) / 4096
    lmax = max(scenes.SUN_COLOR) * O.hg_phase(1.0, 0.6) + 0.2
    assert np.max(np.abs(a - n)) <= xmax / 2 * lmax + 1e-12
    # and the analytic rule at 8 steps is far closer to it than the naive one
    a8 = O.render(vol, cam, replace(p_a, steps=8), 64, 64, pixels=pix)
    n8 = O.render(vol, cam, replace(p_n, steps=8), 64, 64, pixels=pix)
    assert np.abs(a8 - a)[:, :3].mean() < 0.5 * np.abs(n8 - a)[:, :3].mean()


# ---------------------------------------------------------------------------
# Pi6, Pi7: sun on, homogeneous, vertical rays (Sections 1 and 3.1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("N", [1, 2, 8, 128])
@pytest.mark.parametrize("j", [0.0, 0.25, 0.5, 0.9])
def test_front_lit_closed_form(N, j):
    c, alpha, H = 0.1, 10.0, 1.0
    sig = c * alpha
    x = sig * H / N
    Cs, a = np.array(scenes.SUN_COLOR), np.array(scenes.AMBIENT)
    p = params(steps=N, alpha=alpha, sun_dir=(0.0, 1.0, 0.0), g=0.6)
    rgba = one_ray(const_volume(c), (0, 2, 0), (0, -1, 0), p, j)
    P = O.hg_phase(-1.0, 0.6)
    expect = Cs * P * (-math.expm1(-2 * sig * H)) * math.exp(-x * j) / (1 + math.exp(-x)) \
        + a * (-math.expm1(-sig * H))
    assert np.max(np.abs(rgba[:3] - expect)) < 1e-13


@pytest.mark.parametrize("N", [1, 3, 8, 128])
@pytest.mark.parametrize("j", [0.0, 0.5, 0.75])
def test_back_lit_closed_form(N, j):
    c, alpha, H = 0.1, 10.0, 1.0
    sig = c * alpha
    x = sig * H / N
    Cs, a = np.array(scenes.SUN_COLOR), np.array(scenes.AMBIENT)
    p = params(steps=N, alpha=alpha, sun_dir=(0.0, 1.0, 0.0), g=0.6)
    rgba = one_ray(const_volume(c), (0, -2, 0), (0, 1, 0), p, j)
    P = O.hg_phase(1.0, 0.6)
    expect = Cs * P * math.exp(-sig * H) * N * (-math.expm1(-x)) * math.exp(x * j) \
        + a * (-math.expm1(-sig * H))
    assert np.max(np.abs(rgba[:3] - expect)) < 1e-13


def test_light_march_midpoints_and_skip():
    # Linear density along y: the 1-step midpoint rule on a linear profile is
    # exact, so T_L is the exact Beer-Lambert value; rho == 0 skips the march.
    n = 32
    ys = (np.arange(n) + 0.5) / n
    vol = O.OracleVolume(base=np.broadcast_to((0.2 + 0.6 * ys)[None, :, None], (n, n, n)).copy())
    s = np.array([0.0, 1.0, 0.0])
    p = np.array([[0.0, -0.2, 0.0]])
    for L in (1, 2, 6):
        TL = O.light_transmittance(vol, p, s, L, 10.0)[0]
        # integral of 0.2 + 0.6 (y + 0.5) for y in [-0.2, 0.5]
        u0, u1 = 0.3, 1.0
        tau = 10.0 * (0.2 * (u1 - u0) + 0.3 * (u1 ** 2 - u0 ** 2))
        assert TL == pytest.approx(math.exp(-tau), rel=1e-13)
    assert O.light_transmittance(vol, p, s, 0, 10.0)[0] == 1.0


# ---------------------------------------------------------------------------
# Pi8: per-pixel jitter (Section 3.2) averages the step over its length
# ---------------------------------------------------------------------------

def test_jitter_mean_matches_closed_form():
    c, alpha, H, N = 1.0, 10.0, 1.0, 8
    sig = c * alpha
    x = sig * H / N
    py, px = np.meshgrid(np.arange(64), np.arange(64), indexing="ij")
    j = O.jitter_offset(px.reshape(-1), py.reshape(-1), 5, 1609)
    n = j.size
    p = params(steps=N, alpha=alpha, sun_dir=(0.0, 1.0, 0.0), sun_color=(4.0, 0.0, 0.0),
               ambient=(0.0, 0.0, 0.0), jitter=1)
    rgba = O.march_rays(const_volume(c), np.tile([0.0, 2.0, 0.0], (n, 1)),
                        np.tile([0.0, -1.0, 0.0], (n, 1)), p, jitter=j)
    P = O.hg_phase(-1.0, 0.6)
    expect = 4.0 * P * (-math.expm1(-2 * sig * H)) * math.tanh(x / 2) / x
    se = rgba[:, 0].std() / math.sqrt(n)
    assert abs(rgba[:, 0].mean() - expect) < 4 * se
    # the unjittered midpoint value differs from the mean (8 steps keep a bias)
    mid = 4.0 * P * (-math.expm1(-2 * sig * H)) / (2 * math.cosh(x / 2))
    assert abs(mid - expect) > 10 * se


# ---------------------------------------------------------------------------
# Pi10: the jitter hash (reading R14)
# ---------------------------------------------------------------------------

def test_hash_known_answers():
    jit = []
    with open(os.path.join(HERE, "golden", "pcg_kat.txt")) as f:
        for line in f:
            if line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "pcg":
                assert O.pcg_hash(int(parts[1])) == int(parts[2])
                assert int(O.pcg_hash(np.array([int(parts[1])], dtype=np.uint64))[0]) == int(parts[2])
            else:
                px, py, fr, sd, bits = map(int, parts[1:])
                assert O.jitter_offset(px, py, fr, sd) == bits * 2.0 ** -24
                jit.append((px, py, fr, sd, bits))
    # the array path (used by render) gives the same offsets
    for fr, sd in {(r[2], r[3]) for r in jit}:
        rows = [r for r in jit if r[2] == fr and r[3] == sd]
        got = O.jitter_offset(np.array([r[0] for r in rows]), np.array([r[1] for r in rows]), fr, sd)
        assert np.array_equal(got, np.array([r[4] for r in rows]) * 2.0 ** -24)


def test_hash_scalar_matches_vector_and_is_bijective_on_a_range():
    v = np.arange(1 << 20, dtype=np.uint64)
    h = O.pcg_hash(v)
    assert np.unique(h).size == v.size
    for k in (0, 1, 77, 12345, (1 << 20) - 1):
        assert int(h[k]) == O.pcg_hash(k)
    hi = O.pcg_hash(np.array([0xFFFFFFFF, 0x80000000], dtype=np.uint64))
    assert int(hi[0]) == O.pcg_hash(0xFFFFFFFF) and int(hi[1]) == O.pcg_hash(0x80000000)


def test_jitter_uniform():
    from scipy.stats import chi2
    py, px = np.meshgrid(np.arange(1000), np.arange(1000), indexing="ij")
    j = O.jitter_offset(px.reshape(-1), py.reshape(-1), 0, 1609)
    assert j.min() >= 0.0 and j.max() <= 1 - 2 ** -24
    assert abs(j.mean() - 0.5) < 1e-3
    counts = np.bincount((j * 64).astype(np.int64), minlength=64)
    e = j.size / 64
    stat = np.sum((counts - e) ** 2 / e)
    assert chi2.sf(stat, 63) > 1e-3
    # different frames give different offsets for the same pixel
    j1 = O.jitter_offset(px.reshape(-1)[:1000], py.reshape(-1)[:1000], 1, 1609)
    assert np.mean(j1 == j[:1000]) < 0.01


# ---------------------------------------------------------------------------
# Pi11: early-out bound (reading R12)
# ---------------------------------------------------------------------------

def test_early_out_bound():
    rho = scenes.make_density(scenes.WORKLOADS["C1"].volume, cache=False)
    vol = O.OracleVolume(base=rho)
    cam = scenes.orbit_camera(2.0, 210.0, 20.0)
    pix = scenes.random_pixels(64, 64, 400, seed=3)
    for integ in (0, 1):
        p0 = params(steps=64, alpha=60.0, integration=integ, t_eps=0.0)
        p1 = replace(p0, t_eps=1e-5)
        r0, k0 = O.render(vol, cam, p0, 64, 64, pixels=pix, return_lookups=True)
        r1, k1 = O.render(vol, cam, p1, 64, 64, pixels=pix, return_lookups=True)
        lmax = max(scenes.SUN_COLOR) * O.hg_phase(1.0, 0.6) + 0.2
        assert k1 < k0                                   # early-out happened
        assert np.max(np.abs(r0[:, :3] - r1[:, :3])) <= 1e-5 * lmax
        assert np.max(np.abs(r0[:, 3] - r1[:, 3])) <= 1e-5


# ---------------------------------------------------------------------------
# Pi12: temporal resolve (Section 3.2; reading R13)
# ---------------------------------------------------------------------------

def taa_brute(cur, hist, beta):
    H, W, C = cur.shape
    out = np.empty_like(cur)
    for y in range(H):
        for x in range(W):
            for c in range(C):
                nb = [cur[min(max(y + dy, 0), H - 1), min(max(x + dx, 0), W - 1), c]
                      for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
                h = min(max(hist[y, x, c], min(nb)), max(nb))
                out[y, x, c] = h + beta * (cur[y, x, c] - h)
    return out


def test_taa_brute_force_and_frame0():
    rng = np.random.default_rng(4)
    cur, hist = rng.uniform(0, 1, (5, 5, 4)), rng.uniform(-0.5, 1.5, (5, 5, 4))
    out = O.taa_resolve(cur, hist, 0.1, 3)
    assert np.max(np.abs(out - taa_brute(cur, hist, 0.1))) < 1e-15
    assert np.array_equal(O.taa_resolve(cur, hist, 0.1, 0), cur)
    assert np.array_equal(O.taa_resolve(cur, None, 0.1, 4), cur)
    assert np.array_equal(O.taa_resolve(cur, hist, 1.0, 2), cur)


def test_taa_ema_closed_form_and_bounds():
    rng = np.random.default_rng(5)
    cur = rng.uniform(0, 1, (6, 7, 4))
    pad = np.pad(cur, ((1, 1), (1, 1), (0, 0)), mode="edge")
    nb = np.stack([pad[dy:dy + 6, dx:dx + 7] for dy in range(3) for dx in range(3)])
    lo, hi = nb.min(0), nb.max(0)
    h0 = lo + rng.uniform(0, 1, cur.shape) * (hi - lo)   # history inside [m, M]
    h, beta = h0, 0.1
    for k in range(1, 20):
        h = O.taa_resolve(cur, h, beta, k)
        assert np.max(np.abs(h - (cur + (1 - beta) ** k * (h0 - cur)))) < 1e-15
        assert np.all(h >= lo - 1e-15) and np.all(h <= hi + 1e-15)


# ---------------------------------------------------------------------------
# Pi13: brute force on tiny inputs and structural cases
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("integ", [0, 1])
def test_scalar_matches_vectorised(integ):
    rho = scenes.make_density(scenes.WORKLOADS["C1"].volume, cache=False)
    det = scenes.make_detail(8, 33, cache=False)
    cam = scenes.orbit_camera(2.0, 210.0, 20.0)
    pix = scenes.random_pixels(64, 64, 40, seed=9)
    for vol in (O.OracleVolume(base=rho),
                O.OracleVolume(base=rho, detail=det, detail_weight=0.3, detail_tiling=4.0)):
        p = params(steps=32, alpha=8.0, integration=integ, jitter=1, t_eps=1e-5)
        vec = O.render(vol, cam, p, 64, 64, frame=2, pixels=pix)
        o, d = O.camera_rays(cam, 64, 64, pix[:, 0], pix[:, 1])
        j = O.jitter_offset(pix[:, 0], pix[:, 1], 2, p.seed)
        sca = np.array([O.march_ray(vol, o[k], d[k], p, j[k]) for k in range(len(pix))])
        assert np.max(np.abs(vec - sca)) < 1e-14


def test_empty_volume_and_misses_are_exactly_zero():
    cam = scenes.orbit_camera(2.0, 210.0, 20.0)
    p = params(steps=16, jitter=1)
    img = O.render(const_volume(0.0), cam, p, 32, 24)
    assert np.all(img == 0.0)
    rho = scenes.make_density(scenes.WORKLOADS["C1"].volume, cache=False)
    vol = O.OracleVolume(base=rho)
    img, lk = O.render(vol, cam, p, 32, 24, return_lookups=True)
    gx, gy = np.meshgrid(np.arange(32), np.arange(24), indexing="xy")
    o, d = O.camera_rays(cam, 32, 24, gx.reshape(-1), gy.reshape(-1))
    _, _, hit = O.ray_box(o, d, vol.box_min, vol.box_max)
    assert np.all(img.reshape(-1, 4)[~hit] == 0.0)
    assert 0 < hit.mean() < 1
    assert lk >= hit.sum()


def test_mirror_symmetry():
    rho = scenes.make_density(scenes.WORKLOADS["C1"].volume, cache=False)
    sym = 0.5 * (rho + rho[:, :, ::-1])          # symmetric under x -> -x
    vol = O.OracleVolume(base=sym)
    cam = scenes.Camera(pos=(0.0, 0.6, 2.0))       # on the mirror plane x = 0
    p = params(steps=24, jitter=0, sun_dir=(0.0, 0.8, 0.5))
    img = O.render(vol, cam, p, 32, 20)
    assert np.max(np.abs(img - img[:, ::-1])) < 1e-12
    assert img[..., 3].max() > 0.1


# ---------------------------------------------------------------------------
# Lookup trace (which lookups the march performs): against the sample points
# and the early-exit closed form
# ---------------------------------------------------------------------------

def test_trace_light_mask_is_density_positive_at_the_sample_points():
    rho = scenes.make_density(scenes.WORKLOADS["C1"].volume, cache=False)
    vol = O.OracleVolume(base=rho)
    cam = scenes.orbit_camera(2.0, 210.0, 20.0)
    p = params(steps=12, jitter=1, t_eps=0.0)
    W, H = 24, 18
    gx, gy = np.meshgrid(np.arange(W), np.arange(H), indexing="xy")
    px, py = gx.reshape(-1), gy.reshape(-1)
    _, lk, (prim, mask) = O.render(vol, cam, p, W, H, frame=3, pixels=np.stack([px, py], 1),
                                   return_lookups=True, return_trace=True)
    o, d = O.camera_rays(cam, W, H, px, py)
    tn, tf, hit = O.ray_box(o, d, vol.box_min, vol.box_max)
    j = O.jitter_offset(px, py, 3, p.seed)
    # no early exit: every ray through the box takes all N samples
    assert np.array_equal(prim, np.where(hit, p.steps, 0))
    want = np.zeros(px.size, dtype=np.uint64)
    for i in range(p.steps):
        t = tn + (i + j) * (tf - tn) / p.steps
        r = O.density(vol, o + t[:, None] * d)
        want |= np.where(hit & (r > 0), np.uint64(1) << np.uint64(i), np.uint64(0))
    assert np.array_equal(mask, want)
    bits = np.array([bin(int(m)).count("1") for m in mask])
    assert lk == int(prim.sum()) + p.light_steps * int(bits.sum())
    assert 0 < bits.sum() < hit.sum() * p.steps


@pytest.mark.parametrize("alpha,eps", [(10.0, 1e-2), (40.0, 1e-5), (3.0, 1e-5)])
def test_trace_early_exit_closed_form(alpha, eps):
    # homogeneous unit density: T after k samples is exp(-alpha D k), so the
    # march stops after the first k with T < eps (at most N samples)
    vol = const_volume(1.0)
    p = params(steps=16, alpha=alpha, t_eps=eps, light_steps=0)
    o = np.array([[0.0, 0.0, -3.0]])
    d = np.array([[0.0, 0.0, 1.0]])
    _, (prim, mask) = O.march_rays(vol, o, d, p, return_trace=True)
    D = 1.0 / p.steps
    k = np.arange(1, p.steps + 1)
    below = np.nonzero(np.exp(-alpha * D * k) < eps)[0]
    want = int(k[below[0]]) if below.size else p.steps
    assert int(prim[0]) == want
    assert int(mask[0]) == 0      # no light march with light_steps = 0


# ---------------------------------------------------------------------------
# Coherent jitter variants (reading R17): structure, and the same unbiased
# step average over frames as the per-pixel offset
# ---------------------------------------------------------------------------

def test_jitter_modes_structure():
    py, px = np.meshgrid(np.arange(40), np.arange(48), indexing="ij")
    px, py = px.reshape(-1), py.reshape(-1)
    assert O.jitter_for(0, px, py, 3, 1609) is None
    assert np.array_equal(O.jitter_for(1, px, py, 3, 1609), O.jitter_offset(px, py, 3, 1609))
    tile = O.jitter_for(2, px, py, 3, 1609)
    key = (py // 8) * 6 + px // 8
    for k in np.unique(key):
        vals = tile[key == k]
        assert np.all(vals == vals[0])
        assert vals[0] == O.jitter_offset(int(px[key == k][0]) // 8, int(py[key == k][0]) // 8, 3, 1609)
    assert np.unique(tile).size == np.unique(key).size     # 30 tiles, 30 distinct offsets
    frame = O.jitter_for(3, px, py, 3, 1609)
    assert np.all(frame == O.jitter_offset(0, 0, 3, 1609))
    assert O.jitter_for(3, px[:1], py[:1], 4, 1609)[0] != frame[0]
    with pytest.raises(ValueError):
        O.jitter_for(4, px, py, 0, 1)


def test_frame_jitter_mean_over_frames_matches_closed_form():
    # one offset per frame: over many frames the offsets are uniform, so the
    # mean of a ray's colour is the same closed form as the per-pixel mean
    c, alpha, H, N = 1.0, 10.0, 1.0, 8
    sig = c * alpha
    x = sig * H / N
    frames = np.arange(4096)
    j = np.array([O.jitter_for(3, 5, 7, int(f), 1609) for f in frames])
    n = j.size
    p = params(steps=N, alpha=alpha, sun_dir=(0.0, 1.0, 0.0), sun_color=(4.0, 0.0, 0.0),
               ambient=(0.0, 0.0, 0.0), jitter=3)
    rgba = O.march_rays(const_volume(c), np.tile([0.0, 2.0, 0.0], (n, 1)),
                        np.tile([0.0, -1.0, 0.0], (n, 1)), p, jitter=j)
    P = O.hg_phase(-1.0, 0.6)
    expect = 4.0 * P * (-math.expm1(-2 * sig * H)) * math.tanh(x / 2) / x
    se = rgba[:, 0].std() / math.sqrt(n)
    assert abs(rgba[:, 0].mean() - expect) < 4 * se


# ---------------------------------------------------------------------------
# Representative depth and the reprojected resolve (reading R18)
# ---------------------------------------------------------------------------

def test_depth_homogeneous_slab_matches_continuous_mean():
    # opacity-weighted mean distance in a homogeneous slab of length L:
    # int s sigma e^{-sigma s} ds / (1 - e^{-sigma L}) over [0, L]
    for c, alpha in ((1.0, 3.0), (0.5, 1.0), (2.0, 10.0)):
        sig, L = c * alpha, 1.0
        p = params(steps=4096, alpha=alpha, jitter=0, light_steps=0)
        o = np.array([[0.0, 2.0, 0.0]])
        d = np.array([[0.0, -1.0, 0.0]])
        _, depth = O.march_rays(const_volume(c), o, d, p, return_depth=True)
        mean = (1.0 - (1.0 + sig * L) * math.exp(-sig * L)) / (sig * (1.0 - math.exp(-sig * L)))
        assert abs(depth[0] - (1.5 + mean)) < 1e-6


def test_depth_low_alpha_and_misses():
    p = params(steps=16, alpha=1.0, jitter=0, light_steps=0)
    o = np.array([[0.0, 2.0, 0.0], [0.3, 2.0, -0.2], [3.0, 2.0, 0.0]])
    d = np.array([[0.0, -1.0, 0.0], [0.0, -1.0, 0.0], [0.0, -1.0, 0.0]])
    rgba, depth = O.march_rays(const_volume(1e-4), o, d, p, return_depth=True)
    assert rgba[0, 3] < O.DEPTH_ALPHA_MIN
    assert abs(depth[0] - 2.0) < 1e-12 and abs(depth[1] - 2.0) < 1e-12   # chord middle
    assert depth[2] == 0.0                                                   # miss


def test_reproject_with_a_still_camera_is_the_plain_resolve():
    rng = np.random.default_rng(4)
    H, W = 23, 37
    cur, hist = rng.random((H, W, 4)), rng.random((H, W, 4))
    depth = np.where(rng.random((H, W)) < 0.3, 0.0, 1.0 + rng.random((H, W)))
    cam = scenes.orbit_camera(2.0, 210.0, 20.0)
    a = O.taa_resolve_reproject(cur, hist, depth, cam, cam, 0.1, 5)
    b = O.taa_resolve(cur, hist, 0.1, 5)
    assert np.max(np.abs(a - b)) < 1e-10
    assert np.array_equal(O.taa_resolve_reproject(cur, hist, depth, cam, cam, 0.1, 0), cur)


def test_reproject_sideways_translation_samples_the_parallax_shift():
    # camera moved by delta along its right axis since the previous frame: a
    # point at distance z along the view axis moves delta / z in the image
    # plane; bilinear sampling of a linear history is exact inside the image
    H, W, delta, beta = 30, 40, 0.1, 0.25
    cam = scenes.orbit_camera(2.0, 210.0, 20.0)
    pos = np.asarray(cam.pos, float)
    f = np.asarray(cam.target, float) - pos
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(cam.up, float))
    r /= np.linalg.norm(r)
    prev = scenes.Camera(pos=tuple(pos - delta * r), target=tuple(np.asarray(cam.target) - delta * r),
                         up=cam.up, vfov_deg=cam.vfov_deg)
    py, px = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    depth = 1.0 + 0.02 * px + 0.03 * py
    coef = np.array([[0.5, -0.2, 3.0], [0.1, 0.4, -1.0], [-0.3, 0.2, 0.5], [0.05, 0.05, 0.2]])
    hist = np.stack([a * px + b * py + c for a, b, c in coef], axis=-1)
    cur = np.where(((px + py) % 2 == 0)[..., None], 1e6, -1e6) * np.ones(4)
    out = O.taa_resolve_reproject(cur, hist, depth, cam, prev, beta, 3)
    _, d = O.camera_rays(cam, W, H, px.reshape(-1), py.reshape(-1))
    z = depth.reshape(-1) * (d @ f)
    tan_half = math.tan(math.radians(cam.vfov_deg) / 2)
    u = px.reshape(-1) + delta / z * W / (2 * tan_half * W / H)
    w = py.reshape(-1).astype(float)
    inside = u <= W - 1
    want = np.stack([a * u + b * w + c for a, b, c in coef], axis=-1)
    got_h = (out.reshape(-1, 4) - beta * cur.reshape(-1, 4)) / (1 - beta)
    assert np.max(np.abs(got_h[inside] - want[inside])) < 1e-6
    outside = u > W - 0.5
    assert outside.any()
    assert np.array_equal(out.reshape(-1, 4)[outside], cur.reshape(-1, 4)[outside])


# ---------------------------------------------------------------------------
# Composite of the cloud layer into the scene (reading R19)
# ---------------------------------------------------------------------------

def test_composite_same_size_is_the_over_operator():
    rng = np.random.default_rng(8)
    bg = rng.random((9, 13, 4))
    a = rng.random((9, 13, 1))
    cloud = np.concatenate([rng.random((9, 13, 3)) * a, a], axis=-1)
    out = O.composite(cloud, bg)
    # by hand, channel by channel, the over operator for premultiplied colour
    for y, x in ((0, 0), (4, 7), (8, 12)):
        for ch in range(4):
            assert abs(out[y, x, ch] - (cloud[y, x, ch] + (1 - cloud[y, x, 3]) * bg[y, x, ch])) < 1e-15
    clear = np.zeros((9, 13, 4))
    assert np.array_equal(O.composite(clear, bg), bg)
    opaque = cloud.copy()
    opaque[..., 3] = 1.0
    assert np.array_equal(O.composite(opaque, bg), opaque)


@pytest.mark.parametrize("factor", [2, 4])
def test_upsample_linear_field_and_edges(factor):
    h, w = 6, 10
    ly, lx = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    img = np.stack([0.3 * lx + 0.1 * ly, -0.2 * lx + 0.5 * ly, lx * 0 + 1.0, 0.05 * lx], axis=-1)
    up = O.upsample_bilinear(img, w * factor, h * factor)
    Y, X = np.meshgrid(np.arange(h * factor), np.arange(w * factor), indexing="ij")
    u = (X + 0.5) / factor - 0.5
    v = (Y + 0.5) / factor - 0.5
    want = np.stack([0.3 * u + 0.1 * v, -0.2 * u + 0.5 * v, u * 0 + 1.0, 0.05 * u], axis=-1)
    inside = (u >= 0) & (u <= w - 1) & (v >= 0) & (v <= h - 1)
    assert np.max(np.abs(up - want)[inside]) < 1e-12
    # outside the centres of the edge pixels the edge value is held
    left = u < 0
    assert np.allclose(up[left][:, 0], 0.1 * np.clip(v[left], 0, h - 1) + 0.0)
    # a factor-1 resize is the identity
    assert np.array_equal(O.upsample_bilinear(img, w, h), img)

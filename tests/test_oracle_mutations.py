"""Planted mistakes in the oracle must be caught by its pins.

Each case rewrites one line of an oracle function (a dropped term, a wrong
sign or index, a swapped operand, a wrong order of operations), swaps the
mutated function into the oracle module, and checks that at least one of the
pins in test_oracle_pins.py now fails. This runs on the CPU only; the oracle
on disk is never changed.
"""

import inspect
import textwrap

import pytest

import oracle.cloud as OC
from tests import test_oracle_pins as P


def mutated(func_name, old, new):
    src = textwrap.dedent(inspect.getsource(getattr(OC, func_name)))
    assert old in src, f"mutation anchor not found in {func_name}: {old!r}"
    ns = dict(OC.__dict__)
    exec(compile(src.replace(old, new, 1), f"<mutant {func_name}>", "exec"), ns)
    return ns[func_name]


# pins as zero-argument callables
PINS = {
    "hg": lambda: (P.test_hg_normalised_and_mean_cosine(0.6, 64), P.test_hg_spot_values()),
    "camera": lambda: (P.test_camera_single_pixel_looks_at_target(),
                       P.test_camera_field_of_view(65, 33)),
    "box": lambda: P.test_ray_box_cases(),
    "trilinear": lambda: (P.test_trilinear_constant_exact(), P.test_trilinear_linear_in_x_and_clamp(),
                          P.test_trilinear_single_voxel_tent()),
    "detail": lambda: P.test_detail_repeat_and_erosion(),
    "homog": lambda: [P.test_homogeneous_transmittance_and_sun_off(N, j)
                      for N in (3, 8) for j in (0.0, 0.37)],
    "telescope": lambda: P.test_telescoping_any_volume(8),
    "naive": lambda: [P.test_naive_step_dependence_and_convergence(N, r)
                      for N, r in ((8, 0.58198), (16, 0.77075))],
    "front": lambda: [P.test_front_lit_closed_form(N, j) for N in (2, 8) for j in (0.25, 0.9)],
    "back": lambda: [P.test_back_lit_closed_form(N, j) for N in (3, 8) for j in (0.0, 0.75)],
    "light": lambda: P.test_light_march_midpoints_and_skip(),
    "jitter_mean": lambda: P.test_jitter_mean_matches_closed_form(),
    "hash": lambda: (P.test_hash_known_answers(), P.test_jitter_uniform(),
                     P.test_hash_scalar_matches_vector_and_is_bijective_on_a_range()),
    "early": lambda: P.test_early_out_bound(),
    "taa": lambda: (P.test_taa_brute_force_and_frame0(), P.test_taa_ema_closed_form_and_bounds()),
    "mirror": lambda: P.test_mirror_symmetry(),
    "trace": lambda: (P.test_trace_light_mask_is_density_positive_at_the_sample_points(),
                      [P.test_trace_early_exit_closed_form(a, e)
                       for a, e in ((10.0, 1e-2), (40.0, 1e-5))]),
    "jitter_modes": lambda: (P.test_jitter_modes_structure(),
                             P.test_frame_jitter_mean_over_frames_matches_closed_form()),
    "depth": lambda: (P.test_depth_homogeneous_slab_matches_continuous_mean(),
                      P.test_depth_low_alpha_and_misses()),
    "composite": lambda: (P.test_composite_same_size_is_the_over_operator(),
                          [P.test_upsample_linear_field_and_edges(f) for f in (2, 4)]),
    "reproject": lambda: (P.test_reproject_with_a_still_camera_is_the_plain_resolve(),
                          P.test_reproject_sideways_translation_samples_the_parallax_shift()),
}

MUTATIONS = [
    # (name, function, old text, new text)
    ("analytic step uses the updated T", "march_rays",
     "S[idx] += (T[idx] * -np.expm1(-x))[:, None] * L_in\n            T[idx] = T[idx] * np.exp(-x)",
     "T[idx] = T[idx] * np.exp(-x)\n            S[idx] += (T[idx] * -np.expm1(-x))[:, None] * L_in"),
    ("ambient term dropped", "march_rays",
     "L_in = c_sun[None, :] * (phase[idx] * TL)[:, None] + c_amb[None, :]",
     "L_in = c_sun[None, :] * (phase[idx] * TL)[:, None]"),
    ("naive step without the step length", "march_rays",
     "x = rho * alpha * D[idx]", "x = rho * alpha * D[idx] * (1.0 if int(params.integration) == 1 else 1.0 / D[idx].clip(1e-300))"),
    ("jitter offset off by half a step", "march_rays",
     "t = tn[idx] + (i + j[idx]) * D[idx]", "t = tn[idx] + (i + j[idx] - 0.5) * D[idx]"),
    ("step length over N+1", "march_rays",
     "D = np.where(hit, (tf - tn) / N, 0.0)", "D = np.where(hit, (tf - tn) / (N + 1), 0.0)"),
    ("phase with the reversed cosine", "march_rays",
     "phase = hg_phase(d @ s_hat, float(params.g))", "phase = hg_phase(-(d @ s_hat), float(params.g))"),
    ("light transmittance not used", "march_rays",
     "TL[lit] = light_transmittance(vol, p[lit], s_hat, L, alpha)", "TL[lit] = 1.0"),
    ("early exit on the wrong side", "march_rays",
     "alive[idx] = T[idx] >= eps", "alive[idx] = T[idx] >= 10 * eps"),
    ("light samples at step starts", "light_transmittance",
     "q = p + ((k + 0.5) * dl)[:, None] * s_hat[None, :]", "q = p + (k * dl)[:, None] * s_hat[None, :]"),
    ("light optical depth without step length", "light_transmittance",
     "return np.exp(-alpha * dl * acc)", "return np.exp(-alpha * acc / light_steps)"),
    ("light exit towards the wrong face", "light_transmittance",
     "bound = vol.box_max[k] if sk > 0.0 else vol.box_min[k]",
     "bound = vol.box_min[k] if sk > 0.0 else vol.box_max[k]"),
    ("HG without 4 pi", "hg_phase",
     "(4.0 * math.pi * (1.0 + g * g - 2.0 * g", "((1.0 + g * g - 2.0 * g"),
    ("HG with + 2 g mu", "hg_phase",
     "(1.0 + g * g - 2.0 * g", "(1.0 + g * g + 2.0 * g"),
    ("texel corners instead of centres", "density",
     "b = _trilinear(vol.base, uvw[:, 0] * nx - 0.5, uvw[:, 1] * ny - 0.5,",
     "b = _trilinear(vol.base, uvw[:, 0] * nx, uvw[:, 1] * ny - 0.5,"),
    ("x and z swapped in the volume index", "_trilinear",
     "return flat[(z * ny + y) * nx + x]", "return flat[(x * ny + y) * nx + z]"),
    ("lerp weight reversed in y", "_trilinear",
     "return _lerp(_lerp(c00, c10, wy), _lerp(c01, c11, wy), wz)",
     "return _lerp(_lerp(c00, c10, 1 - wy), _lerp(c01, c11, 1 - wy), wz)"),
    ("erosion weight ignored", "density",
     "return np.clip((b - we * d) / (1.0 - we * d), 0.0, 1.0)", "return np.clip(b - we * d, 0.0, 1.0)"),
    ("detail without tiling", "density",
     "d = _trilinear(vol.detail, uvw[:, 0] * t * dx - 0.5", "d = _trilinear(vol.detail, uvw[:, 0] * dx - 0.5"),
    ("slab test ignores the near plane clamp", "ray_box",
     "tn = np.zeros(n)", "tn = np.full(n, -np.inf)"),
    ("vertical FOV used as horizontal", "camera_rays",
     "x = (2.0 * (px + 0.5) / width - 1.0) * tan_half * (width / height)",
     "x = (2.0 * (px + 0.5) / width - 1.0) * tan_half"),
    ("image rows counted from the bottom", "camera_rays",
     "y = (1.0 - 2.0 * (py + 0.5) / height) * tan_half", "y = (2.0 * (py + 0.5) / height - 1.0) * tan_half"),
    ("hash shift off by one", "pcg_hash",
     "w = (((s >> ((s >> 28) + 4)) ^ s) * 277803737) & _M32\n        return ((w >> 22) ^ w).astype(np.uint32)",
     "w = (((s >> ((s >> 28) + 5)) ^ s) * 277803737) & _M32\n        return ((w >> 22) ^ w).astype(np.uint32)"),
    ("jitter keeps the low bits", "jitter_offset",
     "return (h >> 8).astype(np.float64) * 2.0 ** -24", "return (h & 0xFFFFFF).astype(np.float64) * 2.0 ** -24"),
    ("resolve blend reversed", "taa_resolve",
     "return h + blend * (cur - h)", "return cur + blend * (h - cur)"),
    ("resolve without the clamp", "taa_resolve",
     "h = np.minimum(np.maximum(hist, lo), hi)", "h = hist"),
    ("trace records the light march one sample late", "march_rays",
     "mask[idx[lit]] |= np.uint64(1) << np.uint64(i)", "mask[idx[lit]] |= np.uint64(1) << np.uint64(i + 1)"),
    ("tile jitter over 4x4 tiles", "jitter_for",
     "px, py = px >> 3, py >> 3", "px, py = px >> 2, py >> 2"),
    ("depth at the step start", "march_rays",
     "opacity_t[idx] += (T_before - T[idx]) * t", "opacity_t[idx] += (T_before - T[idx]) * (t - j[idx] * D[idx])"),
    ("depth weighted by transmittance", "march_rays",
     "opacity_t[idx] += (T_before - T[idx]) * t", "opacity_t[idx] += T[idx] * t"),
    ("depth of thin rays at the near plane", "march_rays",
     "depth = np.where(a >= DEPTH_ALPHA_MIN, opacity_t / a, 0.5 * (tn + tf))",
     "depth = np.where(a >= DEPTH_ALPHA_MIN, opacity_t / a, tn)"),
    ("reprojection from the current camera", "taa_resolve_reproject",
     "o + dep[:, None] * d - prev_pos[None, :]", "dep[:, None] * d"),
    ("reprojection without the half-pixel shift", "camera_project",
     "uc = (x / (tan_half * (width / height)) + 1.0) * (width * 0.5) - 0.5",
     "uc = (x / (tan_half * (width / height)) + 1.0) * (width * 0.5)"),
    ("bilinear weights swapped", "taa_resolve_reproject",
     "top = _lerp(hist[y0, x0], hist[y0, x1], fx)", "top = _lerp(hist[y0, x0], hist[y0, x1], fy)"),
    ("reprojection off-screen keeps the history", "taa_resolve_reproject",
     "h = np.where(valid[:, None], h, c)", "h = h"),
    ("up-sample with corners aligned", "upsample_bilinear",
     "uc = (np.arange(width) + 0.5) * (w / width) - 0.5", "uc = np.arange(width) * ((w - 1) / max(width - 1, 1))"),
    ("composite weighted by the background alpha", "composite",
     "return c + (1.0 - c[..., 3:4]) * bg", "return c + (1.0 - bg[..., 3:4]) * bg"),
    ("resolve neighbourhood without the edge clamp", "taa_resolve",
     "pad = np.pad(cur, ((1, 1), (1, 1), (0, 0)), mode=\"edge\")",
     "pad = np.pad(cur, ((1, 1), (1, 1), (0, 0)), mode=\"constant\")"),
]


def caught(name):
    for pin in PINS.values():
        try:
            pin()
        except AssertionError:
            return True
    return False


@pytest.mark.parametrize("name,func,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(monkeypatch, name, func, old, new):
    monkeypatch.setattr(OC, func, mutated(func, old, new))
    assert caught(name), f"no pin caught the planted mistake: {name}"


def test_unmutated_oracle_passes_every_pin():
    for pin in PINS.values():
        pin()

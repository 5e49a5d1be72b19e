"""FP64 CPU oracle for the cloud raymarch of Toft, Bowles and Zimmermann,
"Optimisations for Real-Time Volumetric Cloudscapes" (arXiv 1609.05344).

TEST INFRASTRUCTURE ONLY. This package is the slow, plain reference that the
HIP library is checked against. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the library itself never does, and
it shares no code with the library (only the seeded inputs are common).

Every function follows the paper's Section 1 (the raymarch, Beer-Lambert
transmittance, the light march, Henyey-Greenstein phase and ambient term),
Section 3.1 (naive and analytic per-step integration) and Section 3.2 (the
per-pixel jittered start and the temporal accumulation); where the paper is
silent the reading taken is stated at the function.

Parity status: every function is pinned by closed forms, invariants or brute
force in the CPU test suite, except the appearance of full noise-volume images
with the sun on, which only the telescoping invariant (sun off) and the
closed-form slab cases constrain ("parity unpinned" for that combination).
"""

from .cloud import (  # noqa: F401
    OracleVolume,
    pcg_hash,
    jitter_offset,
    hg_phase,
    camera_rays,
    ray_box,
    density,
    light_transmittance,
    march_ray,
    march_rays,
    render,
    taa_resolve,
)

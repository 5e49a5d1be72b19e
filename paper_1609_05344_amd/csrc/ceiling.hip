// Gather-ceiling kernels: the render's density fetches with the arithmetic
// around them removed, to measure what the memory system alone allows for
// the same access pattern and launch shape.
#include <hip/hip_runtime.h>

#include "cloud_device.h"
#include "cloud_launch.h"

namespace cloud {

// The words base_lookup fetches for the footprint at continuous texel
// coordinates f (same clamping, occupancy test and dead-lookup redirect when
// OCC), folded by XOR so that no fetch can be dropped; no decode, no lerps.
template <int DT, int LAYOUT, bool OCC>
__device__ __forceinline__ uint32_t raw_lookup(const DevVolume& v, float fx, float fy, float fz) {
  using S = BaseSampler<DT, LAYOUT>;
  float wx, wy, wz;
  int kx, ky, kz;
  split_coord(fx, v.nx, wx, kx);
  split_coord(fy, v.ny, wy, ky);
  split_coord(fz, v.nz, wz, kz);
  const bool live = OCC ? occupied(v, kx, ky, kz) : true;
  uint32_t w[S::kWords];
  S::load(v, kx, ky, kz, live, w);
  uint32_t x = 0;
#pragma unroll
  for (int k = 0; k < S::kWords; ++k) x ^= w[k];
  return x;
}

// One thread per pixel on the render's tile walk. trace[pixel] = (primary
// samples taken, light-march mask) as recorded by the counting render.
// RANDOM == false: fetch exactly the footprints the render fetches, in the
// same order. RANDOM == true: the same number of lookups per pixel at
// independent uniformly random texel coordinates of the whole volume (no
// occupancy skip). Loop counts are bounded by the step counts whatever the
// trace holds.
template <int DT, int LAYOUT, bool RANDOM>
__global__ __launch_bounds__(256) void gather_ceiling_kernel(DevVolume vol, DevParams prm,
                                                             DevCameras cams, uint32_t frame,
                                                             int W, int H, int tiles_x,
                                                             int tiles_y, int S, int L,
                                                             const uint2* __restrict__ trace,
                                                             float4* __restrict__ out) {
  const int tiles_per_view = tiles_x * tiles_y;
  const int tile = xcd_walk(blockIdx.x, gridDim.x, L);
  const int view = tile / tiles_per_view;
  int tx, ty;
  supertile(tile - view * tiles_per_view, tiles_x, tiles_y, S, tx, ty);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int px, py;
  tile_pixel(tx, ty, wave, lane, px, py);
  stage_volume<LAYOUT>(vol);
  if (px >= W || py >= H) return;
  const size_t pix = ((size_t)view * H + py) * W + px;
  const uint2 tr = trace[pix];
  const uint32_t steps = (uint32_t)prm.steps;   // <= 32 (checked on the host)
  const uint32_t n_prim = min(tr.x, steps);
  const uint32_t mask = steps >= 32 ? tr.y : tr.y & ((1u << steps) - 1u);
  uint32_t acc = 0;
  if constexpr (RANDOM) {
    const uint32_t n = n_prim + (uint32_t)__popc(mask) * (uint32_t)prm.light_steps;
    uint32_t h = pcg((uint32_t)pix + pcg(frame));
    const float sx = (float)vol.nx * 5.9604644775390625e-8f;
    const float sy = (float)vol.ny * 5.9604644775390625e-8f;
    const float sz = (float)vol.nz * 5.9604644775390625e-8f;
    for (uint32_t i = 0; i < n; ++i) {
      // three steps of a 32-bit LCG (Numerical Recipes constants) per point
      h = h * 1664525u + 1013904223u;
      const float fx = fmaf((float)(h >> 8), sx, -0.5f);
      h = h * 1664525u + 1013904223u;
      const float fy = fmaf((float)(h >> 8), sy, -0.5f);
      h = h * 1664525u + 1013904223u;
      const float fz = fmaf((float)(h >> 8), sz, -0.5f);
      acc ^= raw_lookup<DT, LAYOUT, false>(vol, fx, fy, fz);
    }
  } else {
    const DevCamera& c = cams.c[view];
    float dx, dy, dz;
    camera_dir(c, px, py, W, H, dx, dy, dz);
    const float j = jitter_for(prm.jitter, (uint32_t)px, (uint32_t)py, frame, prm.seed);
    const float ox = c.pos[0], oy = c.pos[1], oz = c.pos[2];
    float tn, tf;
    if (n_prim > 0 && ray_box(vol, ox, oy, oz, dx, dy, dz, tn, tf)) {
      const float D = (tf - tn) / (float)prm.steps;
      for (uint32_t i = 0; i < n_prim; ++i) {
        const float t = fmaf((float)i + j, D, tn);
        const float qx = fmaf(t, dx, ox), qy = fmaf(t, dy, oy), qz = fmaf(t, dz, oz);
        acc ^= raw_lookup<DT, LAYOUT, true>(vol, fmaf(qx, vol.sx, vol.ox), fmaf(qy, vol.sy, vol.oy),
                                            fmaf(qz, vol.sz, vol.oz));
        if ((mask >> i) & 1u) {
          const LightPath lp = light_path<false>(vol, prm, qx, qy, qz);
#pragma unroll kLightUnroll
          for (int k = 0; k < prm.light_steps; ++k) {
            const float hk = (float)k + 0.5f;
            acc ^= raw_lookup<DT, LAYOUT, true>(vol, fmaf(hk, lp.dfx, lp.fx0),
                                                fmaf(hk, lp.dfy, lp.fy0), fmaf(hk, lp.dfz, lp.fz0));
          }
        }
      }
    }
  }
  out[pix] = make_float4(__uint_as_float(acc), 0.0f, 0.0f, 0.0f);
}

template <int DT, int LAYOUT>
static hipError_t ceiling_run(const DevVolume& v, const DevParams& p, const DevCameras& c,
                              int n_views, uint32_t frame, int W, int H, const uint32_t* trace,
                              bool random, float* out, hipStream_t s) {
  const int tiles_x = (W + 15) / 16, tiles_y = (H + 15) / 16;
  const dim3 grid(tiles_x * tiles_y * n_views);
  const uint2* tr = reinterpret_cast<const uint2*>(trace);
  float4* o = reinterpret_cast<float4*>(out);
  // as many resident workgroups per CU as the render has (the ceiling needs
  // fewer registers, and more rays in flight would change the cache traffic)
  const void* fn = random ? reinterpret_cast<const void*>(gather_ceiling_kernel<DT, LAYOUT, true>)
                          : reinterpret_cast<const void*>(gather_ceiling_kernel<DT, LAYOUT, false>);
  hipFuncAttributes attr;
  hipError_t e = hipFuncGetAttributes(&attr, fn);
  if (e != hipSuccess) return e;
  const int target = render_residency(DT, LAYOUT, false);
  if (target <= 0) return hipErrorInvalidValue;
  long long pad = residency_lds(target, attr.sharedSizeBytes);
  if (pad < 0) pad = 0;
  const TileWalk tw = tile_walk();
  if (random)
    hipLaunchKernelGGL((gather_ceiling_kernel<DT, LAYOUT, true>), grid, dim3(256), (size_t)pad, s,
                       v, p, c, frame, W, H, tiles_x, tiles_y, tw.S, tw.L, tr, o);
  else
    hipLaunchKernelGGL((gather_ceiling_kernel<DT, LAYOUT, false>), grid, dim3(256), (size_t)pad, s,
                       v, p, c, frame, W, H, tiles_x, tiles_y, tw.S, tw.L, tr, o);
  return hipGetLastError();
}

template <int DT>
static hipError_t ceiling_layout(int layout, const DevVolume& v, const DevParams& p,
                                 const DevCameras& c, int n_views, uint32_t frame, int W, int H,
                                 const uint32_t* trace, bool random, float* out, hipStream_t s) {
  switch (layout) {
    case LAYOUT_QUAD:
      return ceiling_run<DT, LAYOUT_QUAD>(v, p, c, n_views, frame, W, H, trace, random, out, s);
    case LAYOUT_OCT:
      return ceiling_run<DT, LAYOUT_OCT>(v, p, c, n_views, frame, W, H, trace, random, out, s);
    case LAYOUT_QUAD | kLayoutTab:
      return ceiling_run<DT, LAYOUT_QUAD | kLayoutTab>(v, p, c, n_views, frame, W, H, trace, random,
                                                       out, s);
    case LAYOUT_OCT | kLayoutTab:
      return ceiling_run<DT, LAYOUT_OCT | kLayoutTab>(v, p, c, n_views, frame, W, H, trace, random,
                                                      out, s);
    default:
      return ceiling_run<DT, LAYOUT_DENSE>(v, p, c, n_views, frame, W, H, trace, random, out, s);
  }
}

hipError_t launch_ceiling(const DevVolume& v, int dtype, int layout, const DevParams& p,
                          const DevCameras& c, int n_views, uint32_t frame, int W, int H,
                          const uint32_t* trace, bool random, float* out, hipStream_t s) {
  layout = sampler_layout(v, layout);
  switch (dtype) {
    case DT_F16:
      return ceiling_layout<DT_F16>(layout, v, p, c, n_views, frame, W, H, trace, random, out, s);
    case DT_BF16:
      return ceiling_layout<DT_BF16>(layout, v, p, c, n_views, frame, W, H, trace, random, out, s);
    default:
      return ceiling_layout<DT_F32>(layout, v, p, c, n_views, frame, W, H, trace, random, out, s);
  }
}

}  // namespace cloud

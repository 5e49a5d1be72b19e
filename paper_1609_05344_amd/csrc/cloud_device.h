// Device-side building blocks of the cloud raymarch (gfx950).
//
// One thread owns one ray. Nothing here uses floating-point atomics, so every
// output is bitwise reproducible. Storage types are decoded exactly to float32
// and all lerps, optical depths, exponentials and colour run in float32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cloud_types.h"

namespace cloud {

enum { DT_F32 = 0, DT_F16 = 1, DT_BF16 = 2 };

// PCG-RXS-M-XS 32-bit hash (Jarzynski and Olano, JCGT 2020).
__device__ __forceinline__ uint32_t pcg(uint32_t v) {
  uint32_t s = v * 747796405u + 2891336453u;
  uint32_t w = ((s >> ((s >> 28u) + 4u)) ^ s) * 277803737u;
  return (w >> 22u) ^ w;
}

// Per-pixel start offset j in [0, 1) (Section 3.2): hash chain of pixel,
// frame and seed; the top 24 bits scaled by 2^-24 are exact in float32.
__device__ __forceinline__ float jitter_offset(uint32_t px, uint32_t py, uint32_t frame,
                                               uint32_t seed) {
  uint32_t h = pcg(px + pcg(py + pcg(frame + pcg(seed))));
  return (float)(h >> 8) * 5.9604644775390625e-8f;
}

template <int DT>
__device__ __forceinline__ float texel(const void* __restrict__ base, int idx) {
  if constexpr (DT == DT_F32) {
    return static_cast<const float*>(base)[idx];
  } else if constexpr (DT == DT_F16) {
    return (float)static_cast<const _Float16*>(base)[idx];
  } else {
    return __uint_as_float((uint32_t)static_cast<const uint16_t*>(base)[idx] << 16);
  }
}

__device__ __forceinline__ float lerp(float a, float b, float w) { return fmaf(w, b - a, a); }

// Trilinear lookup with clamp-to-edge at continuous texel coordinates
// (x, then y, then z). Coordinates are first bounded to [-1, n], which leaves
// the clamped result unchanged and keeps every index inside the volume for
// any input, NaN included.
template <int DT>
__device__ __forceinline__ float trilerp_clamp(const void* __restrict__ base, int nx, int ny,
                                               int nz, float fx, float fy, float fz) {
  fx = fminf(fmaxf(fx, -1.0f), (float)nx);
  fy = fminf(fmaxf(fy, -1.0f), (float)ny);
  fz = fminf(fmaxf(fz, -1.0f), (float)nz);
  const float x0f = floorf(fx), y0f = floorf(fy), z0f = floorf(fz);
  const float wx = fx - x0f, wy = fy - y0f, wz = fz - z0f;
  const int x0 = (int)x0f, y0 = (int)y0f, z0 = (int)z0f;
  const int xa = min(max(x0, 0), nx - 1), xb = min(max(x0 + 1, 0), nx - 1);
  const int ya = min(max(y0, 0), ny - 1), yb = min(max(y0 + 1, 0), ny - 1);
  const int za = min(max(z0, 0), nz - 1), zb = min(max(z0 + 1, 0), nz - 1);
  const int r00 = (za * ny + ya) * nx, r10 = (za * ny + yb) * nx;
  const int r01 = (zb * ny + ya) * nx, r11 = (zb * ny + yb) * nx;
  const float c00 = lerp(texel<DT>(base, r00 + xa), texel<DT>(base, r00 + xb), wx);
  const float c10 = lerp(texel<DT>(base, r10 + xa), texel<DT>(base, r10 + xb), wx);
  const float c01 = lerp(texel<DT>(base, r01 + xa), texel<DT>(base, r01 + xb), wx);
  const float c11 = lerp(texel<DT>(base, r11 + xa), texel<DT>(base, r11 + xb), wx);
  return lerp(lerp(c00, c10, wy), lerp(c01, c11, wy), wz);
}

// Index k of a periodic axis of n texels, wrapped into [0, n).
__device__ __forceinline__ int wrap_index(int k, int n) {
  int r = k % n;
  return r < 0 ? r + n : r;
}

// Trilinear lookup with repeat addressing (the tiled detail volume).
template <int DT>
__device__ __forceinline__ float trilerp_repeat(const void* __restrict__ base, int nx, int ny,
                                                int nz, float fx, float fy, float fz) {
  const float lim = 1048576.0f;
  fx = fminf(fmaxf(fx, -lim), lim);
  fy = fminf(fmaxf(fy, -lim), lim);
  fz = fminf(fmaxf(fz, -lim), lim);
  const float x0f = floorf(fx), y0f = floorf(fy), z0f = floorf(fz);
  const float wx = fx - x0f, wy = fy - y0f, wz = fz - z0f;
  const int xa = wrap_index((int)x0f, nx), ya = wrap_index((int)y0f, ny),
            za = wrap_index((int)z0f, nz);
  const int xb = xa + 1 == nx ? 0 : xa + 1;
  const int yb = ya + 1 == ny ? 0 : ya + 1;
  const int zb = za + 1 == nz ? 0 : za + 1;
  const int r00 = (za * ny + ya) * nx, r10 = (za * ny + yb) * nx;
  const int r01 = (zb * ny + ya) * nx, r11 = (zb * ny + yb) * nx;
  const float c00 = lerp(texel<DT>(base, r00 + xa), texel<DT>(base, r00 + xb), wx);
  const float c10 = lerp(texel<DT>(base, r10 + xa), texel<DT>(base, r10 + xb), wx);
  const float c01 = lerp(texel<DT>(base, r01 + xa), texel<DT>(base, r01 + xb), wx);
  const float c11 = lerp(texel<DT>(base, r11 + xa), texel<DT>(base, r11 + xb), wx);
  return lerp(lerp(c00, c10, wy), lerp(c01, c11, wy), wz);
}

// Density at world point p (Section 1). With a detail volume the base shape
// is eroded: clamp((b - w d) / (1 - w d), 0, 1); where b <= 0 the result is 0
// whatever d is, so the detail lookup is skipped there.
template <int DT, bool DETAIL>
__device__ __forceinline__ float density(const DevVolume& v, float px, float py, float pz) {
  const float b = trilerp_clamp<DT>(v.base, v.nx, v.ny, v.nz, fmaf(px, v.sx, v.ox),
                                    fmaf(py, v.sy, v.oy), fmaf(pz, v.sz, v.oz));
  if constexpr (!DETAIL) {
    return b;
  } else {
    if (!(b > 0.0f)) return 0.0f;
    const float d = trilerp_repeat<DT>(v.detail, v.dnx, v.dny, v.dnz, fmaf(px, v.dsx, v.dox),
                                       fmaf(py, v.dsy, v.doy), fmaf(pz, v.dsz, v.doz));
    const float wd = v.detail_weight * d;
    return fminf(fmaxf((b - wd) / (1.0f - wd), 0.0f), 1.0f);
  }
}

// Transmittance towards the sun from p (Section 1): L midpoint samples of
// equal steps up to the box exit along s, Beer-Lambert over their sum.
template <int DT, bool DETAIL>
__device__ __forceinline__ float light_transmittance(const DevVolume& v, const DevParams& P,
                                                     float px, float py, float pz) {
  float tx = 3.402823466e38f;
  if (P.s_axis[0]) tx = fminf(tx, (P.light_bound[0] - px) * P.inv_s[0]);
  if (P.s_axis[1]) tx = fminf(tx, (P.light_bound[1] - py) * P.inv_s[1]);
  if (P.s_axis[2]) tx = fminf(tx, (P.light_bound[2] - pz) * P.inv_s[2]);
  const float dl = tx * P.inv_light_steps;
  const float stx = dl * P.s[0], sty = dl * P.s[1], stz = dl * P.s[2];
  float acc = 0.0f;
  for (int k = 0; k < P.light_steps; ++k) {
    const float h = (float)k + 0.5f;
    acc += density<DT, DETAIL>(v, fmaf(h, stx, px), fmaf(h, sty, py), fmaf(h, stz, pz));
  }
  return exp2f(-P.alpha_log2e * dl * acc);
}

struct RayResult {
  float r, g, b, a;
};

// One primary ray through the volume (Sections 1, 3.1, 3.2). (o, d): origin
// and unit direction; j: start offset in [0, 1).
template <int DT, bool DETAIL, int INTEG>
__device__ __forceinline__ RayResult march(const DevVolume& v, const DevParams& P, float ox,
                                           float oy, float oz, float dx, float dy, float dz,
                                           float j) {
  RayResult res = {0.0f, 0.0f, 0.0f, 0.0f};
  // slab test; an axis with d_k == 0 passes iff the origin lies in the slab
  float tn = 0.0f, tf = 3.402823466e38f;
  bool hit = true;
  const float o3[3] = {ox, oy, oz}, d3[3] = {dx, dy, dz};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (d3[k] == 0.0f) {
      hit = hit && (o3[k] >= v.bmin[k]) && (o3[k] <= v.bmax[k]);
    } else {
      const float inv = 1.0f / d3[k];
      const float t0 = (v.bmin[k] - o3[k]) * inv, t1 = (v.bmax[k] - o3[k]) * inv;
      tn = fmaxf(tn, fminf(t0, t1));
      tf = fminf(tf, fmaxf(t0, t1));
    }
  }
  if (!hit || !(tf > tn)) return res;

  const float D = (tf - tn) / (float)P.steps;
  const float mu = dx * P.s[0] + dy * P.s[1] + dz * P.s[2];
  const float q = fmaf(-P.hg_b, mu, P.hg_a);
  const float phase = P.hg_k / (q * sqrtf(q));
  const float sr = P.sun[0] * phase, sg = P.sun[1] * phase, sb = P.sun[2] * phase;
  const float kx = P.alpha_log2e * D;   // exp2 scale of rho for one step

  float T = 1.0f, Sr = 0.0f, Sg = 0.0f, Sb = 0.0f;
  for (int i = 0; i < P.steps; ++i) {
    const float t = fmaf((float)i + j, D, tn);
    const float px = fmaf(t, dx, ox), py = fmaf(t, dy, oy), pz = fmaf(t, dz, oz);
    const float rho = density<DT, DETAIL>(v, px, py, pz);
    if (rho > 0.0f) {
      const float TL = P.light_steps > 0 ? light_transmittance<DT, DETAIL>(v, P, px, py, pz) : 1.0f;
      const float lr = fmaf(sr, TL, P.amb[0]), lg = fmaf(sg, TL, P.amb[1]),
                  lb = fmaf(sb, TL, P.amb[2]);
      const float e = exp2f(-rho * kx);
      if constexpr (INTEG == 1) {
        const float w = T * (1.0f - e);
        Sr = fmaf(w, lr, Sr);
        Sg = fmaf(w, lg, Sg);
        Sb = fmaf(w, lb, Sb);
        T *= e;
      } else {
        T *= e;
        const float w = T * (rho * P.alpha * D);
        Sr = fmaf(w, lr, Sr);
        Sg = fmaf(w, lg, Sg);
        Sb = fmaf(w, lb, Sb);
      }
      if (T < P.t_eps) break;
    }
  }
  res.r = Sr;
  res.g = Sg;
  res.b = Sb;
  res.a = 1.0f - T;
  return res;
}

// Unit view direction through the centre of pixel (px, py).
__device__ __forceinline__ void camera_dir(const DevCamera& c, int px, int py, int W, int H,
                                           float& dx, float& dy, float& dz) {
  const float x = (2.0f * ((float)px + 0.5f) / (float)W - 1.0f) * c.tan_half * c.aspect;
  const float y = (1.0f - 2.0f * ((float)py + 0.5f) / (float)H) * c.tan_half;
  float ux = c.fwd[0] + x * c.right[0] + y * c.up[0];
  float uy = c.fwd[1] + x * c.right[1] + y * c.up[1];
  float uz = c.fwd[2] + x * c.right[2] + y * c.up[2];
  const float inv = rsqrtf(ux * ux + uy * uy + uz * uz);
  dx = ux * inv;
  dy = uy * inv;
  dz = uz * inv;
}

// Block index -> tile index so that each XCD (workgroups are dealt to the 8
// XCDs round-robin) receives one contiguous run of tiles, keeping neighbouring
// tiles -- which read the same part of the volume -- in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int x = b & 7, k = b >> 3;
  return x * q + min(x, r) + k;
}

}  // namespace cloud

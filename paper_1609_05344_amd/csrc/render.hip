// Render, explicit-ray and temporal-resolve kernels, and their launchers.
#include <hip/hip_runtime.h>

#include "cloud_device.h"
#include "cloud_launch.h"

namespace cloud {

// ---------------------------------------------------------------------------
// cloud_render / cloud_render_views: one thread per pixel. A 256-thread
// workgroup covers a 16x16 pixel tile as four 8x8 wave tiles, so the 64 rays
// of a wavefront are a compact bundle that samples neighbouring texels.
// ---------------------------------------------------------------------------

template <int DT, bool DETAIL, int INTEG>
__global__ __launch_bounds__(256) void render_kernel(DevVolume vol, DevParams prm,
                                                     DevCameras cams, uint32_t frame, int W,
                                                     int H, int tiles_x, int tiles_per_view,
                                                     float4* __restrict__ out) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int view = tile / tiles_per_view;
  const int t = tile - view * tiles_per_view;
  const int ty = t / tiles_x, tx = t - ty * tiles_x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int px = tx * 16 + (wave & 1) * 8 + (lane & 7);
  const int py = ty * 16 + (wave >> 1) * 8 + (lane >> 3);
  if (px >= W || py >= H) return;

  const DevCamera& c = cams.c[view];
  float dx, dy, dz;
  camera_dir(c, px, py, W, H, dx, dy, dz);
  const float j = prm.jitter ? jitter_offset((uint32_t)px, (uint32_t)py, frame, prm.seed) : 0.5f;
  const RayResult r = march<DT, DETAIL, INTEG>(vol, prm, c.pos[0], c.pos[1], c.pos[2], dx, dy,
                                               dz, j);
  out[((size_t)view * H + py) * W + px] = make_float4(r.r, r.g, r.b, r.a);
}

template <int DT, bool DETAIL, int INTEG>
__global__ __launch_bounds__(256) void rays_kernel(DevVolume vol, DevParams prm, uint32_t frame,
                                                   const float* __restrict__ origins,
                                                   const float* __restrict__ dirs,
                                                   const uint32_t* __restrict__ pixel_xy,
                                                   long long n, float4* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float ox = origins[3 * i], oy = origins[3 * i + 1], oz = origins[3 * i + 2];
  float dx = dirs[3 * i], dy = dirs[3 * i + 1], dz = dirs[3 * i + 2];
  const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
  dx *= inv;
  dy *= inv;
  dz *= inv;
  float j = 0.5f;
  if (prm.jitter && pixel_xy) j = jitter_offset(pixel_xy[2 * i], pixel_xy[2 * i + 1], frame, prm.seed);
  const RayResult r = march<DT, DETAIL, INTEG>(vol, prm, ox, oy, oz, dx, dy, dz, j);
  out[i] = make_float4(r.r, r.g, r.b, r.a);
}

// ---------------------------------------------------------------------------
// Temporal resolve (Section 3.2): a 16x16 tile of the current frame plus a
// one-pixel edge-clamped halo is staged in LDS, so each current pixel is read
// from HBM once although nine threads use it.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void taa_kernel(const float4* __restrict__ cur,
                                                  const float4* hist, float4* out, int W, int H,
                                                  int tiles_x, float blend) {
  __shared__ float4 tile[18][18];
  const int tyi = blockIdx.x / tiles_x, txi = blockIdx.x - tyi * tiles_x;
  const int bx = txi * 16, by = tyi * 16;
  for (int i = threadIdx.x; i < 18 * 18; i += 256) {
    const int ly = i / 18, lx = i - ly * 18;
    const int gx = min(max(bx + lx - 1, 0), W - 1);
    const int gy = min(max(by + ly - 1, 0), H - 1);
    tile[ly][lx] = cur[(size_t)gy * W + gx];
  }
  __syncthreads();
  const int lx = threadIdx.x & 15, ly = threadIdx.x >> 4;
  const int px = bx + lx, py = by + ly;
  if (px >= W || py >= H) return;
  const float4 c = tile[ly + 1][lx + 1];
  float4 lo = c, hi = c;
#pragma unroll
  for (int dy = 0; dy < 3; ++dy) {
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      const float4 v = tile[ly + dy][lx + dx];
      lo.x = fminf(lo.x, v.x); lo.y = fminf(lo.y, v.y); lo.z = fminf(lo.z, v.z); lo.w = fminf(lo.w, v.w);
      hi.x = fmaxf(hi.x, v.x); hi.y = fmaxf(hi.y, v.y); hi.z = fmaxf(hi.z, v.z); hi.w = fmaxf(hi.w, v.w);
    }
  }
  const size_t p = (size_t)py * W + px;
  float4 h = hist[p];
  h.x = fminf(fmaxf(h.x, lo.x), hi.x);
  h.y = fminf(fmaxf(h.y, lo.y), hi.y);
  h.z = fminf(fmaxf(h.z, lo.z), hi.z);
  h.w = fminf(fmaxf(h.w, lo.w), hi.w);
  out[p] = make_float4(fmaf(blend, c.x - h.x, h.x), fmaf(blend, c.y - h.y, h.y),
                       fmaf(blend, c.z - h.z, h.z), fmaf(blend, c.w - h.w, h.w));
}

__global__ __launch_bounds__(256) void jitter_kernel(const uint32_t* __restrict__ pxy, long long n,
                                                     uint32_t frame, uint32_t seed,
                                                     uint32_t* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (uint32_t)(jitter_offset(pxy[2 * i], pxy[2 * i + 1], frame, seed) * 16777216.0f);
}

__global__ __launch_bounds__(256) void copy_kernel(const float4* __restrict__ src,
                                                   float4* __restrict__ dst, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

template <int DT, bool DETAIL, int INTEG>
static hipError_t launch_render_t(const DevVolume& v, const DevParams& p, const DevCameras& c,
                                  int n_views, uint32_t frame, int W, int H, float* out,
                                  hipStream_t s) {
  const int tiles_x = (W + 15) / 16, tiles_y = (H + 15) / 16;
  const int tiles_per_view = tiles_x * tiles_y;
  const int blocks = tiles_per_view * n_views;
  hipLaunchKernelGGL((render_kernel<DT, DETAIL, INTEG>), dim3(blocks), dim3(256), 0, s, v, p, c,
                     frame, W, H, tiles_x, tiles_per_view, reinterpret_cast<float4*>(out));
  return hipGetLastError();
}

template <int DT, bool DETAIL, int INTEG>
static hipError_t launch_rays_t(const DevVolume& v, const DevParams& p, uint32_t frame,
                                const float* o, const float* d, const uint32_t* pxy, long long n,
                                float* out, hipStream_t s) {
  const long long blocks = (n + 255) / 256;
  hipLaunchKernelGGL((rays_kernel<DT, DETAIL, INTEG>), dim3((unsigned)blocks), dim3(256), 0, s,
                     v, p, frame, o, d, pxy, n, reinterpret_cast<float4*>(out));
  return hipGetLastError();
}

#define CLOUD_DISPATCH(FN, dt, detail, integ, ...)                                 \
  do {                                                                             \
    if (dt == DT_F32) {                                                            \
      if (detail) return integ ? FN<DT_F32, true, 1>(__VA_ARGS__)                  \
                               : FN<DT_F32, true, 0>(__VA_ARGS__);                 \
      return integ ? FN<DT_F32, false, 1>(__VA_ARGS__) : FN<DT_F32, false, 0>(__VA_ARGS__); \
    } else if (dt == DT_F16) {                                                     \
      if (detail) return integ ? FN<DT_F16, true, 1>(__VA_ARGS__)                  \
                               : FN<DT_F16, true, 0>(__VA_ARGS__);                 \
      return integ ? FN<DT_F16, false, 1>(__VA_ARGS__) : FN<DT_F16, false, 0>(__VA_ARGS__); \
    } else {                                                                       \
      if (detail) return integ ? FN<DT_BF16, true, 1>(__VA_ARGS__)                 \
                               : FN<DT_BF16, true, 0>(__VA_ARGS__);                \
      return integ ? FN<DT_BF16, false, 1>(__VA_ARGS__) : FN<DT_BF16, false, 0>(__VA_ARGS__); \
    }                                                                              \
  } while (0)

hipError_t launch_render(const DevVolume& v, int dtype, const DevParams& p, const DevCameras& c,
                         int n_views, uint32_t frame, int W, int H, float* out, hipStream_t s) {
  const bool detail = v.detail != nullptr;
  CLOUD_DISPATCH(launch_render_t, dtype, detail, p.integration, v, p, c, n_views, frame, W, H,
                 out, s);
}

hipError_t launch_rays(const DevVolume& v, int dtype, const DevParams& p, uint32_t frame,
                       const float* o, const float* d, const uint32_t* pxy, long long n,
                       float* out, hipStream_t s) {
  const bool detail = v.detail != nullptr;
  CLOUD_DISPATCH(launch_rays_t, dtype, detail, p.integration, v, p, frame, o, d, pxy, n, out, s);
}

hipError_t launch_jitter(const uint32_t* pxy, long long n, uint32_t frame, uint32_t seed,
                         uint32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(jitter_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pxy, n,
                     frame, seed, out);
  return hipGetLastError();
}

hipError_t launch_taa(const float* cur, const float* hist, float* out, int W, int H, float blend,
                      bool copy, hipStream_t s) {
  if (copy) {
    const long long n = (long long)W * H;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<const float4*>(cur), reinterpret_cast<float4*>(out), n);
    return hipGetLastError();
  }
  const int tiles_x = (W + 15) / 16, tiles_y = (H + 15) / 16;
  hipLaunchKernelGGL(taa_kernel, dim3(tiles_x * tiles_y), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(cur), reinterpret_cast<const float4*>(hist),
                     reinterpret_cast<float4*>(out), W, H, tiles_x, blend);
  return hipGetLastError();
}

}  // namespace cloud

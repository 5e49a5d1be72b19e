// Temporal resolve kernels and their launcher.
#include <hip/hip_runtime.h>

#include "cloud_launch.h"

namespace cloud {

// ---------------------------------------------------------------------------
// Temporal resolve (Section 3.2): a tile of 256 pixels of the current frame
// (TW wide) plus a one-pixel edge-clamped halo is staged in LDS, so each
// current pixel is read from HBM about once although nine threads use it.
// ---------------------------------------------------------------------------

template <int TW>
__global__ __launch_bounds__(256) void taa_kernel(const float4* __restrict__ cur,
                                                  const float4* hist, float4* out, int W, int H,
                                                  int tiles_x, float blend) {
  constexpr int TH = 256 / TW;
  __shared__ float4 tile[TH + 2][TW + 2];
  const int tyi = blockIdx.x / tiles_x, txi = blockIdx.x - tyi * tiles_x;
  const int bx = txi * TW, by = tyi * TH;
  for (int i = threadIdx.x; i < (TH + 2) * (TW + 2); i += 256) {
    const int ly = i / (TW + 2), lx = i - ly * (TW + 2);
    const int gx = min(max(bx + lx - 1, 0), W - 1);
    const int gy = min(max(by + ly - 1, 0), H - 1);
    tile[ly][lx] = cur[(size_t)gy * W + gx];
  }
  __syncthreads();
  const int lx = threadIdx.x % TW, ly = threadIdx.x / TW;
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

__global__ __launch_bounds__(256) void copy_kernel(const float4* __restrict__ src,
                                                   float4* __restrict__ dst, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

hipError_t launch_taa(const float* cur, const float* hist, float* out, int W, int H, float blend,
                      bool copy, hipStream_t s) {
  if (copy) {
    const long long n = (long long)W * H;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<const float4*>(cur), reinterpret_cast<float4*>(out), n);
    return hipGetLastError();
  }
  const float4* c4 = reinterpret_cast<const float4*>(cur);
  const float4* h4 = reinterpret_cast<const float4*>(hist);
  float4* o4 = reinterpret_cast<float4*>(out);
  const int tw = tuning().taa_tile;
  const int th = 256 / tw;
  const int tiles_x = (W + tw - 1) / tw, tiles_y = (H + th - 1) / th;
  const dim3 grid(tiles_x * tiles_y);
  if (tw == 64)
    hipLaunchKernelGGL(taa_kernel<64>, grid, dim3(256), 0, s, c4, h4, o4, W, H, tiles_x, blend);
  else if (tw == 32)
    hipLaunchKernelGGL(taa_kernel<32>, grid, dim3(256), 0, s, c4, h4, o4, W, H, tiles_x, blend);
  else
    hipLaunchKernelGGL(taa_kernel<16>, grid, dim3(256), 0, s, c4, h4, o4, W, H, tiles_x, blend);
  return hipGetLastError();
}

}  // namespace cloud

// Composite of the resolved cloud layer into the scene (Section 3.2: the
// clouds are rendered and resolved in a low-resolution buffer that is then
// composited into the rest of the frame).
#include <hip/hip_runtime.h>

#include "cloud_launch.h"

namespace cloud {

__device__ __forceinline__ float4 mix4(float4 a, float4 b, float w) {
  return make_float4(fmaf(w, b.x - a.x, a.x), fmaf(w, b.y - a.y, a.y), fmaf(w, b.z - a.z, a.z),
                     fmaf(w, b.w - a.w, a.w));
}

// One thread per output pixel, blocks of 256 along an image row (coalesced
// background and output). The layer is sampled bilinearly with pixel centres
// aligned (output x samples the layer at (x + 1/2) lw / W - 1/2, edge-clamped);
// neighbouring threads share the layer's texels through the caches.
__global__ __launch_bounds__(256) void composite_kernel(const float4* __restrict__ layer, int lw,
                                                        int lh, const float4* bg, float4* out,
                                                        int W, int row_blocks, float sx,
                                                        float sy) {
  const int y = blockIdx.x / row_blocks;
  const int x = (blockIdx.x - y * row_blocks) * 256 + threadIdx.x;
  if (x >= W) return;
  const float uc = fmaf((float)x + 0.5f, sx, -0.5f);
  const float vc = fmaf((float)y + 0.5f, sy, -0.5f);
  const float x0f = floorf(uc), y0f = floorf(vc);
  const float fx = uc - x0f, fy = vc - y0f;
  const int x0 = (int)x0f, y0 = (int)y0f;   // >= -1
  const int xa = min(max(x0, 0), lw - 1), xb = min(max(x0 + 1, 0), lw - 1);
  const int ya = min(max(y0, 0), lh - 1), yb = min(max(y0 + 1, 0), lh - 1);
  const float4 top = mix4(layer[(size_t)ya * lw + xa], layer[(size_t)ya * lw + xb], fx);
  const float4 bot = mix4(layer[(size_t)yb * lw + xa], layer[(size_t)yb * lw + xb], fx);
  const float4 c = mix4(top, bot, fy);
  const size_t p = (size_t)y * W + x;
  const float4 b = bg[p];
  const float t = 1.0f - c.w;
  out[p] = make_float4(fmaf(t, b.x, c.x), fmaf(t, b.y, c.y), fmaf(t, b.z, c.z), fmaf(t, b.w, c.w));
}

hipError_t launch_composite(const float* layer, int lw, int lh, const float* bg, float* out, int W,
                            int H, hipStream_t s) {
  const int row_blocks = (W + 255) / 256;
  hipLaunchKernelGGL(composite_kernel, dim3(row_blocks * H), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(layer), lw, lh,
                     reinterpret_cast<const float4*>(bg), reinterpret_cast<float4*>(out), W,
                     row_blocks, (float)lw / (float)W, (float)lh / (float)H);
  return hipGetLastError();
}

}  // namespace cloud

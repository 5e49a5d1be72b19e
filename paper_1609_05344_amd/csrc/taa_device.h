// One tile of the temporal resolve (Section 3.2), shared by the resolve
// kernel and the fused render-and-resolve kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "stream_io.h"

namespace cloud {

// Tile t (row-major, tiles_x a row) of TW x (R * 256 / TW) pixels, R pixels
// a thread (rows r, r + 256 / TW, ... of the tile): the tile of the current
// frame plus a one-pixel edge-clamped halo is staged in LDS, so each current
// pixel is read from memory about once although nine threads use it; each
// pixel's history is clamped into its 3x3 neighbourhood's per-channel range
// and blended towards the current value. More pixels a thread put more loads
// in flight a wavefront, for a kernel whose register allocation holds few
// wavefronts. Every thread of the workgroup must call it (it holds a
// barrier).
// tile is the LDS staging area, (R * 256 / TW + 2) rows of TW + 2 pixels.
template <int TW, int R>
__device__ __forceinline__ void taa_block_rows(float4 (*tile)[TW + 2], int t,
                                               const float4* __restrict__ cur, const float4* hist,
                                               float4* out, int W, int H, int tiles_x,
                                               float blend) {
  constexpr int TH = R * 256 / TW;
  const int tyi = t / tiles_x, txi = t - tyi * tiles_x;
  const int bx = txi * TW, by = tyi * TH;
  for (int i = threadIdx.x; i < (TH + 2) * (TW + 2); i += 256) {
    const int ly = i / (TW + 2), lx = i - ly * (TW + 2);
    const int gx = min(max(bx + lx - 1, 0), W - 1);
    const int gy = min(max(by + ly - 1, 0), H - 1);
    tile[ly][lx] = cur[(size_t)gy * W + gx];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int lx = threadIdx.x % TW, ly = threadIdx.x / TW + r * (TH / R);
    const int px = bx + lx, py = by + ly;
    if (px >= W || py >= H) continue;
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
    float4 h = load_stream(hist + p);
    h.x = fminf(fmaxf(h.x, lo.x), hi.x);
    h.y = fminf(fmaxf(h.y, lo.y), hi.y);
    h.z = fminf(fmaxf(h.z, lo.z), hi.z);
    h.w = fminf(fmaxf(h.w, lo.w), hi.w);
    store_stream(out + p, make_float4(fmaf(blend, c.x - h.x, h.x), fmaf(blend, c.y - h.y, h.y),
                                      fmaf(blend, c.z - h.z, h.z), fmaf(blend, c.w - h.w, h.w)));
  }
}


// One pixel a thread: tiles of 256 pixels, TW wide, staged in an LDS array
// of their own.
template <int TW>
__device__ __forceinline__ void taa_block(int t, const float4* __restrict__ cur, const float4* hist,
                                          float4* out, int W, int H, int tiles_x, float blend) {
  __shared__ float4 tile[256 / TW + 2][TW + 2];
  taa_block_rows<TW, 1>(tile, t, cur, hist, out, W, H, tiles_x, blend);
}

}  // namespace cloud

// Launch-ready forms of the ABI structs (host and device).
//
// The host side folds everything that is uniform over a launch -- texel
// scaling, the normalised sun direction, light-exit planes, phase constants,
// the camera basis -- into these structs once per call, so the kernels do no
// per-pixel set-up beyond the ray itself.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cloud {

constexpr int kMaxViews = 16;   // cameras carried by value in one launch

// Base-volume layouts. All hold the same texel values; the packed ones
// replicate each lookup's footprint so that it is one aligned fetch.
enum { LAYOUT_DENSE = 0, LAYOUT_QUAD = 1, LAYOUT_OCT = 2 };

// Entry order of the packed layouts: 1 (default) bricks of 2x2x2 entries --
// one 128-byte line of 16-byte entries -- with the bricks row-major, so that a
// line holds a small cube of footprints and a quad lookup's two planes share
// a line half the time; 0 row-major [z][y][x] entries. Renders are bitwise the
// same either way; only the addresses differ.
#ifndef CLOUD_SWIZZLE
#define CLOUD_SWIZZLE 1
#endif

// Product of two non-negative ints below 2^24 (plane strides are checked
// against that on the host): the full-rate 24-bit multiply on the device.
inline __host__ __device__ int mul24(int a, int b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul24(a, b);
#else
  return a * b;
#endif
}

// Index of packed entry (x, y, z) given the row and plane strides (entries
// per row and per plane, or bricks per brick row and brick plane).
inline __host__ __device__ int packed_index(int x, int y, int z, int row, int plane) {
#if CLOUD_SWIZZLE
  return ((mul24(z >> 1, plane) + mul24(y >> 1, row) + (x >> 1)) << 3) | ((z & 1) << 2) |
         ((y & 1) << 1) | (x & 1);
#else
  return mul24(z, plane) + mul24(y, row) + x;
#endif
}

// Strides and entry count of a packed layout of ex x ey x ez entries.
inline __host__ __device__ void packed_strides(long long ex, long long ey, long long ez,
                                               long long* row, long long* plane,
                                               long long* entries) {
#if CLOUD_SWIZZLE
  const long long bx = (ex + 1) / 2, by = (ey + 1) / 2, bz = (ez + 1) / 2;
  *row = bx;
  *plane = bx * by;
  *entries = bx * by * bz * 8;
#else
  *row = ex;
  *plane = ex * ey;
  *entries = ex * ey * ez;
#endif
}

struct DevVolume {
  const void* base;
  int nx, ny, nz;
  int plane;            // dense: nx * ny; packed: the plane stride of packed_index
  int row;              // dense: nx; packed: the row stride of packed_index
  // continuous texel coordinate along each axis: f = p * s + o, texel k's
  // centre at f = k (texel centres at box_min + (k + 0.5) * extent / n)
  float sx, sy, sz, ox, oy, oz;
  const void* detail;           // dense, or oct-wrap packed when the base is packed
  int dnx, dny, dnz;
  int dpow2;                    // every detail dim is a power of two
  float dsx, dsy, dsz, dox, doy, doz;
  float detail_weight;
  float bmin[3], bmax[3];
  // occupancy bitmap (nullptr = none): bricks of 2^occ_lg texels per axis
  const uint32_t* occ;
  int occ_lg, occ_nbx, occ_nby, occ_words;
};

constexpr int kOccupancyWords = 1024;   // LDS budget of the bitmap (32768 bricks)

struct DevParams {
  int steps, light_steps;
  float alpha;          // extinction per unit density
  float alpha_log2e;    // alpha * log2(e), for exp2
  float inv_light_steps;
  float s[3];           // unit direction towards the sun
  float light_bound[3]; // exit plane per axis along s (box_max if s_k > 0)
  float inv_s[3];       // 1 / s_k
  int s_axis[3];        // s_k != 0
  float sun[3], amb[3];
  float hg_k;           // (1 - g^2) / (4 pi)
  float hg_a, hg_b;     // 1 + g^2, 2 g
  int jitter;
  uint32_t seed;
  int integration;
  float t_eps;
};

struct DevCamera {
  float pos[3];
  float fwd[3], right[3], up[3];
  float tan_half, aspect;   // tan(vfov/2), width/height
};

struct DevCameras {
  DevCamera c[kMaxViews];
};

}  // namespace cloud

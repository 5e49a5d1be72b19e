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

// A packed entry index is the sum of a term of x, a term of y and a term of
// z (see packed_index), and so is its byte offset. For a volume of at most
// kTabAxis texels along x and y, fewer along z, and below 4 GiB stored, the
// kernels stage those byte-offset terms in LDS tables and index through them;
// the sampler's layout argument then carries kLayoutTab.
constexpr int kLayoutTab = 4;
constexpr int kTabAxis = 1024;
inline __host__ __device__ bool tab_fits(int nx, int ny, int nz) {
  return nx <= kTabAxis && ny <= kTabAxis && nz < kTabAxis;
}

// Entry order of the packed layouts: bricks of 2^bx x 2^by x 2^bz entries --
// 8 in all, one 128-byte line of 16-byte entries -- x fastest inside a brick,
// then y, then z, with the bricks themselves row-major. The shape is a
// property of the packed volume (default 2 x 2 x 2: a small cube of
// footprints per line, and a quad lookup's two planes share a line half the
// time). Renders are bitwise the same for every shape; only addresses differ.

// Product of two non-negative ints below 2^24 (plane strides are checked
// against that on the host): the full-rate 24-bit multiply on the device.
inline __host__ __device__ int mul24(int a, int b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul24(a, b);
#else
  return a * b;
#endif
}

// Index of packed entry (x, y, z) for brick shifts (bx, by, bz) and the
// brick-row and brick-plane strides.
inline __host__ __device__ int packed_index(int x, int y, int z, int bx, int by, int bz, int row,
                                            int plane) {
  return ((mul24(z >> bz, plane) + mul24(y >> by, row) + (x >> bx)) << 3) |
         ((z & ((1 << bz) - 1)) << (bx + by)) | ((y & ((1 << by) - 1)) << bx) |
         (x & ((1 << bx) - 1));
}

// Strides (bricks per brick row and per brick plane) and the stored entry
// count of a packed layout of ex x ey x ez entries in bricks (bx, by, bz).
inline __host__ __device__ void packed_strides(long long ex, long long ey, long long ez, int bx,
                                               int by, int bz, long long* row, long long* plane,
                                               long long* entries) {
  const long long nbx = (ex + (1 << bx) - 1) >> bx, nby = (ey + (1 << by) - 1) >> by;
  const long long nbz = (ez + (1 << bz) - 1) >> bz;
  *row = nbx;
  *plane = nbx * nby;
  *entries = nbx * nby * nbz * 8;
}

struct DevVolume {
  const void* base;
  int nx, ny, nz;
  int plane;            // dense: nx * ny; packed: the plane stride of packed_index
  int row;              // dense: nx; packed: the row stride of packed_index
  int bx, by, bz;       // packed: brick shifts of packed_index
  int entry_shift;      // packed: log2 of an entry's bytes (quad 4, oct 8 texels)
  int tab;              // packed and indexed through the LDS byte-offset tables
  uint32_t tab_bytes;   // with tab: the stored bytes (the buffer range of its fetches)
  // continuous texel coordinate along each axis: f = p * s + o, texel k's
  // centre at f = k (texel centres at box_min + (k + 0.5) * extent / n)
  float sx, sy, sz, ox, oy, oz;
  const void* detail;           // dense, or oct-wrap packed when the base is packed
  int dnx, dny, dnz;
  int dpow2;                    // every detail dim is a power of two
  float dsx, dsy, dsz, dox, doy, doz;
  float detail_weight;
  float bmin[3], bmax[3];
  // occupancy bitmap (nullptr = none): bricks of 2^occ_lg texels per axis,
  // occ_nbx per brick row and occ_plane per brick plane
  const uint32_t* occ;
  int occ_lg, occ_nbx, occ_plane, occ_words;
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

// Launch-ready forms of the ABI structs (host and device).
//
// The host side folds everything that is uniform over a launch -- texel
// scaling, the normalised sun direction, light-exit planes, phase constants,
// the camera basis -- into these structs once per call, so the kernels do no
// per-pixel set-up beyond the ray itself.
#pragma once

#include <stdint.h>

namespace cloud {

constexpr int kMaxViews = 16;   // cameras carried by value in one launch

// Base-volume layouts. All hold the same texel values; the packed ones
// replicate each lookup's footprint so that it is one aligned fetch.
enum { LAYOUT_DENSE = 0, LAYOUT_QUAD = 1, LAYOUT_OCT = 2 };

struct DevVolume {
  const void* base;
  int nx, ny, nz;
  int plane;            // dense: nx * ny; packed: (nx + 1) * (ny + 1) entries
  int row;              // dense: nx; packed: nx + 1 entries
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

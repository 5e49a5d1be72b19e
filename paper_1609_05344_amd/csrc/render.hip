// Render, explicit-ray, lookup-count, volume-pack and temporal-resolve
// kernels, and their launchers.
#include <hip/hip_runtime.h>

#include <mutex>

#include "cloud_device.h"
#include "cloud_launch.h"
#include "taa_device.h"

namespace cloud {

Tuning& tuning() {
  static Tuning t;
  return t;
}

// Default: 4 x 4 super-tiles, one per XCD run. Of the shapes measured (S in
// 4..8, runs of 16..256 tiles, at 480x270 to 8 x 3840x2160) it was best or
// within 3 % of best everywhere; longer runs leave fewer rounds to even out
// the XCDs' shares at the smaller sizes, and some lengths alias with the
// image width so that an XCD keeps landing on the same columns.
TileWalk tile_walk() {
  const Tuning& t = tuning();
  const int S = t.supertile >= 0 ? t.supertile : 4;
  const int L = t.xcd_run >= 0 ? t.xcd_run : S * S;
  return {S, L};
}

// ---------------------------------------------------------------------------
// cloud_render / cloud_render_views / cloud_count_lookups: one thread per
// pixel. A 256-thread workgroup covers a 16x16 pixel tile as four 8x8 wave
// tiles, so the 64 rays of a wavefront are a compact bundle that samples
// neighbouring texels. MODE kImage stores the image; kCount adds up the
// density lookups (into counts, if given) and records each pixel's (primary
// samples, light-march mask) pair (into trace, if given) instead; kDepth
// stores the image and each pixel's representative depth (into depth).
// ---------------------------------------------------------------------------

enum { kImage = 0, kCount = 1, kDepth = 2 };

// Block b of a render of nb tile blocks (b names the XCD as b % 8).
template <int DT, int LAYOUT, bool DETAIL, int MODE>
__device__ __forceinline__ void render_block(int b, int nb, const DevVolume& vol,
                                             const DevParams& prm, const DevCameras& cams,
                                             uint32_t frame, int W, int H, int tiles_x,
                                             int tiles_y, int S, int L, float4* __restrict__ out,
                                             unsigned long long* __restrict__ counts,
                                             uint2* __restrict__ trace,
                                             float* __restrict__ depth) {
  constexpr bool COUNT = MODE == kCount;
  const int tiles_per_view = tiles_x * tiles_y;
  // On odd frames each XCD takes its blocks in reverse order (blocks x,
  // x + 8, ... are XCD x's), so a frame starts on the tiles each XCD ended
  // the one before with, whose volume lines its L2 and the last-level cache
  // still hold.
  if (frame & 1u) {
    const int x = b & 7, k = b >> 3, nx = (nb - x + 7) >> 3;
    b = 8 * (nx - 1 - k) + x;
  }
  const int tile = xcd_walk(b, nb, L);
  const int view = tile / tiles_per_view;
  int tx, ty;
  supertile(tile - view * tiles_per_view, tiles_x, tiles_y, S, tx, ty);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int px, py;
  tile_pixel(tx, ty, wave, lane, px, py);
  const bool inside = px < W && py < H;
  // the ray's set-up runs while the occupancy bitmap is on its way to LDS
  StagedOccupancy staged;
  stage_volume_begin(vol, staged);
  const DevCamera& c = cams.c[view];
  float dx = 0.0f, dy = 0.0f, dz = 1.0f, j = 0.5f;
  if (inside) {
    camera_dir(c, px, py, W, H, dx, dy, dz);
    j = jitter_for(prm.jitter, (uint32_t)px, (uint32_t)py, frame, prm.seed);
  }
  stage_volume_end<LAYOUT>(vol, staged);
  if (!COUNT && !inside) return;

  RayResult r = {0.0f, 0.0f, 0.0f, 0.0f, 0u, 0u, 0u, 0.0f};
  if (inside)
    r = march<DT, LAYOUT, DETAIL, COUNT, MODE == kDepth>(vol, prm, c.pos[0], c.pos[1], c.pos[2],
                                                         dx, dy, dz, j);
  if constexpr (COUNT) {
    if (counts) {
      const uint32_t s = wave_sum(r.lookups);
      if (lane == 0) atomicAdd(counts, (unsigned long long)s);
    }
    if (trace && inside) trace[((size_t)view * H + py) * W + px] = make_uint2(r.primary, r.light_mask);
  } else {
    const size_t pix = ((size_t)view * H + py) * W + px;
    out[pix] = make_float4(r.r, r.g, r.b, r.a);
    if constexpr (MODE == kDepth) depth[pix] = r.depth;
  }
}

template <int DT, int LAYOUT, bool DETAIL, int MODE>
__global__ __launch_bounds__(256) void render_kernel(DevVolume vol, DevParams prm,
                                                     DevCameras cams, uint32_t frame, int W,
                                                     int H, int tiles_x, int tiles_y, int S,
                                                     int L, float4* __restrict__ out,
                                                     unsigned long long* __restrict__ counts,
                                                     uint2* __restrict__ trace,
                                                     float* __restrict__ depth) {
  render_block<DT, LAYOUT, DETAIL, MODE>(blockIdx.x, gridDim.x, vol, prm, cams, frame, W, H,
                                         tiles_x, tiles_y, S, L, out, counts, trace, depth);
}

// The fused kernel's resolve takes two pixels a thread (32 x 16 tiles): its
// workgroups carry the render's register allocation, so fewer of them fit a
// CU than of the plain resolve's, and each needs more loads in flight.
constexpr int kFusedRows = 2;

// The render of frame f and the resolve of frame f - 1 of n_views views in
// one launch (cloud_render_resolve): blocks [0, nbp) render (nb of them are
// tiles; nbp rounds nb up to a multiple of 8, so that the resolve's blocks
// keep block % 8 as their XCD), the rest resolve prev against hist into
// resolved, view by view ([n_views][H][W] images; taa_tiles a view), or copy
// prev there when copy is set. The resolve's blocks come last, so they fill
// the render's tail, when fewer and fewer of its tiles are left.
template <int DT, int LAYOUT, bool DETAIL>
__global__ __launch_bounds__(256) void render_resolve_kernel(
    DevVolume vol, DevParams prm, DevCameras cams, uint32_t frame, int W, int H, int tiles_x,
    int tiles_y, int S, int L, float4* __restrict__ out, int nb, int nbp,
    const float4* __restrict__ prev, const float4* hist, float4* resolved, int taa_tiles_x,
    int taa_tiles, int n_views, float blend, int xcd_runs, int copy) {
  if ((int)blockIdx.x < nbp) {
    if ((int)blockIdx.x < nb)
      render_block<DT, LAYOUT, DETAIL, kImage>(blockIdx.x, nb, vol, prm, cams, frame, W, H,
                                               tiles_x, tiles_y, S, L, out, nullptr, nullptr,
                                               nullptr);
    return;
  }
  const int t = (int)blockIdx.x - nbp;
  if (copy) {
    // 256 pixels of the n_views images, in memory order
    const long long i = (long long)t * 256 + threadIdx.x;
    if (i < (long long)n_views * W * H) resolved[i] = prev[i];
    return;
  }
  const int tt = xcd_runs ? xcd_walk(t, taa_tiles * n_views, 0) : t;
  const int view = tt / taa_tiles;
  const size_t o = (size_t)view * W * H;
  // the resolve's tile is staged in the render's table area: a workgroup
  // runs one part or the other, so the launch holds no more LDS than a render
  constexpr int TH = kFusedRows * 256 / 32;
  static_assert(sizeof(float4) * (TH + 2) * 34 <= sizeof(s_terms), "resolve tile exceeds the tables");
  taa_block_rows<32, kFusedRows>(reinterpret_cast<float4(*)[34]>(s_terms), tt - view * taa_tiles,
                                 prev + o, hist + o, resolved + o, W, H, taa_tiles_x, blend);
}

template <int DT, int LAYOUT, bool DETAIL>
__global__ __launch_bounds__(256) void rays_kernel(DevVolume vol, DevParams prm, uint32_t frame,
                                                   const float* __restrict__ origins,
                                                   const float* __restrict__ dirs,
                                                   const uint32_t* __restrict__ pixel_xy,
                                                   long long n, float4* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  stage_volume<LAYOUT>(vol);
  if (i >= n) return;
  const float ox = origins[3 * i], oy = origins[3 * i + 1], oz = origins[3 * i + 2];
  float dx = dirs[3 * i], dy = dirs[3 * i + 1], dz = dirs[3 * i + 2];
  const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
  dx *= inv;
  dy *= inv;
  dz *= inv;
  float j = 0.5f;
  if (pixel_xy) j = jitter_for(prm.jitter, pixel_xy[2 * i], pixel_xy[2 * i + 1], frame, prm.seed);
  const RayResult r = march<DT, LAYOUT, DETAIL, false>(vol, prm, ox, oy, oz, dx, dy, dz, j);
  out[i] = make_float4(r.r, r.g, r.b, r.a);
}

// ---------------------------------------------------------------------------
// Volume packing: entry (z', y', x') of a packed layout holds the texels of
// the corner k = (x'-1, y'-1, z'-1) and its +1 neighbours, edge-clamped
// (quad: x and y only, plane z = z'). Storage values are copied bit for bit.
// ---------------------------------------------------------------------------

template <typename E, int CORNERS>
__global__ __launch_bounds__(256) void pack_kernel(const E* __restrict__ src, int nx, int ny,
                                                   int nz, int ez, int bx, int by, int bz,
                                                   int row, int plane, E* __restrict__ dst) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long ex = nx + 1, ey = ny + 1;
  if (e >= ex * ey * ez) return;
  const int ix = (int)(e % ex), iy = (int)((e / ex) % ey), iz = (int)(e / (ex * ey));
  const int x = ix - 1;
  const int y = iy - 1;
  const int z = iz - (CORNERS == 8 ? 1 : 0);
  const int xa = min(max(x, 0), nx - 1), xb = min(max(x + 1, 0), nx - 1);
  const int ya = min(max(y, 0), ny - 1), yb = min(max(y + 1, 0), ny - 1);
  const int za = min(max(z, 0), nz - 1), zb = min(max(z + 1, 0), nz - 1);
  const size_t pa = (size_t)za * ny * nx, pb = (size_t)zb * ny * nx;
  E* o = dst + (size_t)packed_index(ix, iy, iz, bx, by, bz, row, plane) * CORNERS;
  o[0] = src[pa + (size_t)ya * nx + xa];
  o[1] = src[pa + (size_t)ya * nx + xb];
  o[2] = src[pa + (size_t)yb * nx + xa];
  o[3] = src[pa + (size_t)yb * nx + xb];
  if constexpr (CORNERS == 8) {
    o[4] = src[pb + (size_t)ya * nx + xa];
    o[5] = src[pb + (size_t)ya * nx + xb];
    o[6] = src[pb + (size_t)yb * nx + xa];
    o[7] = src[pb + (size_t)yb * nx + xb];
  }
}

// Detail packing (repeat addressing): entry (z, y, x) holds the texels at
// x|x+1, y|y+1, z|z+1, each wrapped, in the oct order.
template <typename E>
__global__ __launch_bounds__(256) void pack_wrap_kernel(const E* __restrict__ src, int nx, int ny,
                                                        int nz, E* __restrict__ dst) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)nx * ny * nz) return;
  const int x = (int)(e % nx), y = (int)((e / nx) % ny), z = (int)(e / ((long long)nx * ny));
  const int x1 = x + 1 == nx ? 0 : x + 1, y1 = y + 1 == ny ? 0 : y + 1, z1 = z + 1 == nz ? 0 : z + 1;
  const size_t p0 = (size_t)z * ny * nx, p1 = (size_t)z1 * ny * nx;
  E* o = dst + (size_t)e * 8;
  o[0] = src[p0 + (size_t)y * nx + x];
  o[1] = src[p0 + (size_t)y * nx + x1];
  o[2] = src[p0 + (size_t)y1 * nx + x];
  o[3] = src[p0 + (size_t)y1 * nx + x1];
  o[4] = src[p1 + (size_t)y * nx + x];
  o[5] = src[p1 + (size_t)y * nx + x1];
  o[6] = src[p1 + (size_t)y1 * nx + x];
  o[7] = src[p1 + (size_t)y1 * nx + x1];
}

// ---------------------------------------------------------------------------
// Occupancy bitmap: bit b is set when brick b -- texels [k, k + 2^lg] per
// axis (one texel past the brick, so every footprint whose corner lies in the
// brick is covered), clamped to the volume -- holds a non-zero texel.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void fill_zero_kernel(uint32_t* __restrict__ out, int words) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < words) out[i] = 0u;
}

template <typename E>
__global__ __launch_bounds__(256) void occupancy_kernel(const E* __restrict__ src, int nx, int ny,
                                                        int nz, int lg, int nbx, int nby, int nbz,
                                                        E magnitude_mask,
                                                        uint32_t* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbx * nby * nbz) return;
  const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
  const int x0 = bx << lg, y0 = by << lg, z0 = bz << lg;
  const int x1 = min(x0 + (1 << lg), nx - 1), y1 = min(y0 + (1 << lg), ny - 1),
            z1 = min(z0 + (1 << lg), nz - 1);
  bool any = false;
  for (int z = z0; z <= z1 && !any; ++z)
    for (int y = y0; y <= y1 && !any; ++y)
      for (int x = x0; x <= x1; ++x)
        if (src[((size_t)z * ny + y) * nx + x] & magnitude_mask) {
          any = true;
          break;
        }
  if (any) atomicOr(&out[b >> 5], 1u << (b & 31));
}

__global__ __launch_bounds__(256) void jitter_kernel(const uint32_t* __restrict__ pxy, long long n,
                                                     uint32_t frame, uint32_t seed,
                                                     uint32_t* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (uint32_t)(jitter_offset(pxy[2 * i], pxy[2 * i + 1], frame, seed) * 16777216.0f);
}


// ---------------------------------------------------------------------------
// Launchers: runtime (dtype, layout, detail, count) -> template instance
// ---------------------------------------------------------------------------

template <typename F, int DT, int LAYOUT, bool DETAIL>
static hipError_t dispatch_m(int mode, F& f) {
  switch (mode) {
    case kCount: return f.template run<DT, LAYOUT, DETAIL, kCount>();
    case kDepth: return f.template run<DT, LAYOUT, DETAIL, kDepth>();
    default: return f.template run<DT, LAYOUT, DETAIL, kImage>();
  }
}

template <typename F, int DT, int LAYOUT>
static hipError_t dispatch_dc(bool detail, int mode, F& f) {
  return detail ? dispatch_m<F, DT, LAYOUT, true>(mode, f) : dispatch_m<F, DT, LAYOUT, false>(mode, f);
}

template <typename F, int DT>
static hipError_t dispatch_l(int layout, bool detail, int mode, F& f) {
  switch (layout) {
    case LAYOUT_QUAD: return dispatch_dc<F, DT, LAYOUT_QUAD>(detail, mode, f);
    case LAYOUT_OCT: return dispatch_dc<F, DT, LAYOUT_OCT>(detail, mode, f);
    case LAYOUT_QUAD | kLayoutTab: return dispatch_dc<F, DT, LAYOUT_QUAD | kLayoutTab>(detail, mode, f);
    case LAYOUT_OCT | kLayoutTab: return dispatch_dc<F, DT, LAYOUT_OCT | kLayoutTab>(detail, mode, f);
    default: return dispatch_dc<F, DT, LAYOUT_DENSE>(detail, mode, f);
  }
}

template <typename F>
static hipError_t dispatch(int dtype, int layout, bool detail, int mode, F& f) {
  switch (dtype) {
    case DT_F16: return dispatch_l<F, DT_F16>(layout, detail, mode, f);
    case DT_BF16: return dispatch_l<F, DT_BF16>(layout, detail, mode, f);
    default: return dispatch_l<F, DT_F32>(layout, detail, mode, f);
  }
}

// LDS bytes per CU and per workgroup of device dev (cached; false on error).
static bool lds_limits(int dev, int* per_cu, int* per_block) {
  constexpr int kDevs = 64;
  static std::mutex mu;
  static int cu[kDevs], blk[kDevs];
  if (dev < 0 || dev >= kDevs) return false;
  std::lock_guard<std::mutex> lock(mu);
  if (!cu[dev]) {
    int a = 0, b = 0;
    if (hipDeviceGetAttribute(&a, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) !=
            hipSuccess ||
        hipDeviceGetAttribute(&b, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        a <= 0 || b <= 0)
      return false;
    cu[dev] = a;
    blk[dev] = b;
  }
  *per_cu = cu[dev];
  *per_block = blk[dev];
  return true;
}

template <typename K>
static size_t static_lds_of(K fn) {
  hipFuncAttributes a;
  return hipFuncGetAttributes(&a, reinterpret_cast<const void*>(fn)) == hipSuccess
             ? a.sharedSizeBytes
             : kOccupancyWords * 4;
}

long long residency_lds(int blocks_per_cu, size_t static_lds) {
  if (blocks_per_cu <= 0) return 0;
  int dev = 0, per_cu = 0, per_block = 0;
  if (hipGetDevice(&dev) != hipSuccess || !lds_limits(dev, &per_cu, &per_block)) return -1;
  // blocks_per_cu + 1 workgroups of (static + dynamic) bytes must not fit
  long long total = (long long)per_cu / (blocks_per_cu + 1) + 1;
  total = (total + 255) & ~255LL;
  if ((long long)blocks_per_cu * total > per_cu || total > per_block) return -1;
  return total > (long long)static_lds ? total - (long long)static_lds : 0;
}

// The residency cap in force for a render of this dtype and layout.
template <int DT, int LAYOUT>
static int render_cap() {
  return tuning().render_blocks_per_cu;
}

struct RenderLaunch {
  const DevVolume& v;
  const DevParams& p;
  const DevCameras& c;
  int n_views;
  uint32_t frame;
  int W, H;
  float* out;
  unsigned long long* counts;
  uint32_t* trace;
  float* depth;
  hipStream_t s;
  template <int DT, int LAYOUT, bool DETAIL, int MODE>
  hipError_t run() {
    const int tiles_x = (W + 15) / 16, tiles_y = (H + 15) / 16;
    const int tiles_per_view = tiles_x * tiles_y;
    const int blocks = tiles_per_view * n_views;
    size_t lds = 0;
    if (MODE != kCount && render_cap<DT, LAYOUT>() > 0) {
      static const size_t slds = static_lds_of(render_kernel<DT, LAYOUT, DETAIL, MODE>);
      const long long pad = residency_lds(render_cap<DT, LAYOUT>(), slds);
      if (pad < 0) return hipErrorInvalidValue;
      lds = (size_t)pad;
    }
    const TileWalk tw = tile_walk();
    hipLaunchKernelGGL((render_kernel<DT, LAYOUT, DETAIL, MODE>), dim3(blocks), dim3(256), lds, s,
                       v, p, c, frame, W, H, tiles_x, tiles_y, tw.S, tw.L,
                       reinterpret_cast<float4*>(out), counts, reinterpret_cast<uint2*>(trace),
                       depth);
    return hipGetLastError();
  }
};

struct RenderResolveLaunch {
  const DevVolume& v;
  const DevParams& p;
  const DevCameras& c;
  int n_views;
  uint32_t frame;
  int W, H;
  float* out;
  const float* prev;
  const float* hist;
  float* resolved;
  float blend;
  bool copy;
  hipStream_t s;
  template <int DT, int LAYOUT, bool DETAIL, int MODE>
  hipError_t run() {
    if constexpr (MODE != kImage) {
      return hipErrorInvalidValue;
    } else {
      const int tiles_x = (W + 15) / 16, tiles_y = (H + 15) / 16;
      const int nb = tiles_x * tiles_y * n_views, nbp = (nb + 7) / 8 * 8;
      constexpr int TW = 32, TH = kFusedRows * 256 / TW;   // taa_block_rows's tiles
      const int ttx = (W + TW - 1) / TW, tty = (H + TH - 1) / TH;
      const long long px = (long long)W * H * n_views;
      const long long taa_blocks = copy ? (px + 255) / 256 : (long long)ttx * tty * n_views;
      const TileWalk tw = tile_walk();
      hipLaunchKernelGGL((render_resolve_kernel<DT, LAYOUT, DETAIL>),
                         dim3((unsigned)(nbp + taa_blocks)), dim3(256), 0, s, v, p, c, frame, W, H,
                         tiles_x, tiles_y, tw.S, tw.L, reinterpret_cast<float4*>(out), nb, nbp,
                         reinterpret_cast<const float4*>(prev),
                         reinterpret_cast<const float4*>(hist),
                         reinterpret_cast<float4*>(resolved), ttx, ttx * tty, n_views, blend,
                         taa_xcd_runs(W, H * n_views), copy ? 1 : 0);
      return hipGetLastError();
    }
  }
};

struct RaysLaunch {
  const DevVolume& v;
  const DevParams& p;
  uint32_t frame;
  const float *o, *d;
  const uint32_t* pxy;
  long long n;
  float* out;
  hipStream_t s;
  template <int DT, int LAYOUT, bool DETAIL, int MODE>
  hipError_t run() {
    const long long blocks = (n + 255) / 256;
    hipLaunchKernelGGL((rays_kernel<DT, LAYOUT, DETAIL>), dim3((unsigned)blocks), dim3(256), 0, s,
                       v, p, frame, o, d, pxy, n, reinterpret_cast<float4*>(out));
    return hipGetLastError();
  }
};

hipError_t launch_render(const DevVolume& v, int dtype, int layout, const DevParams& p,
                         const DevCameras& c, int n_views, uint32_t frame, int W, int H,
                         float* out, unsigned long long* counts, uint32_t* trace,
                         float* depth, hipStream_t s) {
  RenderLaunch f{v, p, c, n_views, frame, W, H, out, counts, trace, depth, s};
  const int mode = counts != nullptr || trace != nullptr ? kCount : depth != nullptr ? kDepth : kImage;
  return dispatch(dtype, sampler_layout(v, layout), v.detail != nullptr, mode, f);
}

hipError_t launch_render_resolve(const DevVolume& v, int dtype, int layout, const DevParams& p,
                                 const DevCameras& c, int n_views, uint32_t frame, int W, int H,
                                 float* out, const float* prev, const float* hist,
                                 float* resolved, float blend, bool copy, hipStream_t s) {
  RenderResolveLaunch f{v, p, c, n_views, frame, W, H, out, prev, hist, resolved, blend, copy, s};
  return dispatch(dtype, sampler_layout(v, layout), v.detail != nullptr, kImage, f);
}

hipError_t launch_rays(const DevVolume& v, int dtype, int layout, const DevParams& p,
                       uint32_t frame, const float* o, const float* d, const uint32_t* pxy,
                       long long n, float* out, hipStream_t s) {
  RaysLaunch f{v, p, frame, o, d, pxy, n, out, s};
  return dispatch(dtype, sampler_layout(v, layout), v.detail != nullptr, kImage, f);
}

hipError_t launch_pack(const void* src, int elem_bytes, int nx, int ny, int nz, int layout,
                       const int* brick, void* dst, hipStream_t s) {
  const int ez = layout == LAYOUT_OCT ? nz + 1 : nz;
  const long long entries = (long long)(nx + 1) * (ny + 1) * ez;
  const unsigned blocks = (unsigned)((entries + 255) / 256);
  long long row, plane, stored;
  const int bx = brick[0], by = brick[1], bz = brick[2];
  packed_strides(nx + 1, ny + 1, ez, bx, by, bz, &row, &plane, &stored);
  if (elem_bytes == 4) {
    if (layout == LAYOUT_OCT)
      hipLaunchKernelGGL((pack_kernel<uint32_t, 8>), dim3(blocks), dim3(256), 0, s,
                         static_cast<const uint32_t*>(src), nx, ny, nz, ez, bx, by, bz, (int)row, (int)plane,
                         static_cast<uint32_t*>(dst));
    else
      hipLaunchKernelGGL((pack_kernel<uint32_t, 4>), dim3(blocks), dim3(256), 0, s,
                         static_cast<const uint32_t*>(src), nx, ny, nz, ez, bx, by, bz, (int)row, (int)plane,
                         static_cast<uint32_t*>(dst));
  } else {
    if (layout == LAYOUT_OCT)
      hipLaunchKernelGGL((pack_kernel<uint16_t, 8>), dim3(blocks), dim3(256), 0, s,
                         static_cast<const uint16_t*>(src), nx, ny, nz, ez, bx, by, bz, (int)row, (int)plane,
                         static_cast<uint16_t*>(dst));
    else
      hipLaunchKernelGGL((pack_kernel<uint16_t, 4>), dim3(blocks), dim3(256), 0, s,
                         static_cast<const uint16_t*>(src), nx, ny, nz, ez, bx, by, bz, (int)row, (int)plane,
                         static_cast<uint16_t*>(dst));
  }
  return hipGetLastError();
}

hipError_t launch_pack_detail(const void* src, int elem_bytes, int nx, int ny, int nz, void* dst,
                              hipStream_t s) {
  const long long n = (long long)nx * ny * nz;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (elem_bytes == 4)
    hipLaunchKernelGGL((pack_wrap_kernel<uint32_t>), dim3(blocks), dim3(256), 0, s,
                       static_cast<const uint32_t*>(src), nx, ny, nz, static_cast<uint32_t*>(dst));
  else
    hipLaunchKernelGGL((pack_wrap_kernel<uint16_t>), dim3(blocks), dim3(256), 0, s,
                       static_cast<const uint16_t*>(src), nx, ny, nz, static_cast<uint16_t*>(dst));
  return hipGetLastError();
}

hipError_t launch_occupancy(const void* src, int elem_bytes, int nx, int ny, int nz, int lg,
                            int nbx, int nby, int nbz, uint32_t* out, hipStream_t s) {
  const int bricks = nbx * nby * nbz, words = (bricks + 31) / 32;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((words + 255) / 256), dim3(256), 0, s, out, words);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned blocks = (unsigned)((bricks + 255) / 256);
  if (elem_bytes == 4)
    hipLaunchKernelGGL((occupancy_kernel<uint32_t>), dim3(blocks), dim3(256), 0, s,
                       static_cast<const uint32_t*>(src), nx, ny, nz, lg, nbx, nby, nbz,
                       (uint32_t)0x7FFFFFFFu, out);
  else
    hipLaunchKernelGGL((occupancy_kernel<uint16_t>), dim3(blocks), dim3(256), 0, s,
                       static_cast<const uint16_t*>(src), nx, ny, nz, lg, nbx, nby, nbz,
                       (uint16_t)0x7FFFu, out);
  return hipGetLastError();
}

hipError_t launch_jitter(const uint32_t* pxy, long long n, uint32_t frame, uint32_t seed,
                         uint32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(jitter_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pxy, n,
                     frame, seed, out);
  return hipGetLastError();
}

}  // namespace cloud

// Gather record and replay: the render's own density fetches replayed
// without the arithmetic around them, a measurement of the render's access
// pattern on its own (the per-pixel jitter's cost is cache misses, Sections 4
// and 5).
//
// Two kernels. gather_record_kernel walks the render's rays once (untimed)
// and writes every lookup the render makes as the texel corner of its
// footprint, in the order the wavefront issues them: slot s of wavefront w is
// one lookup instruction of that wavefront, 64 codes wide (one per lane, a
// sentinel for lanes that take no part in it). gather_replay_kernel then
// fetches, per wavefront and slot, the words those corners address, with no
// camera, jitter, ray-box, light-path, interpolation or lighting arithmetic:
// a coalesced code load, the corner decode, the layout's entry index, the
// fetch.
#include <hip/hip_runtime.h>

#include "cloud_device.h"
#include "cloud_launch.h"

namespace cloud {

// code: kx | ky << 10 | kz << 20 | dead << 30; kReplaySkip for a lane that
// makes no lookup in the slot. dead: the occupancy skip redirects the fetch
// to entry 0 (the render's empty-brick lookup).
constexpr uint32_t kReplaySkip = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t corner_code(const DevVolume& v, float fx, float fy, float fz) {
  float wx, wy, wz;
  int kx, ky, kz;
  split_coord(fx, v.nx, wx, kx);
  split_coord(fy, v.ny, wy, ky);
  split_coord(fz, v.nz, wz, kz);
  const bool live = occupied(v, kx, ky, kz);
  return (uint32_t)kx | ((uint32_t)ky << 10) | ((uint32_t)kz << 20) | (live ? 0u : 1u << 30);
}

// Global wavefront index of (tile, wave): the tile's index in the render's
// block order (view-major), four wavefronts a tile.
__device__ __forceinline__ size_t wave_index(int tile, int wave) { return (size_t)tile * 4 + wave; }

// One thread per pixel on the render's launch shape and tile walk. trace:
// per pixel (primary samples taken, light-march mask), from
// cloud_lookup_trace. A wavefront takes its slots in the render's order:
// step i's primary lookup while any lane is still marching, then the L light
// lookups if any lane ran the light march at step i. The step loop is
// bounded by params.steps whatever trace holds, so at most
// steps * (1 + light_steps) <= max_slots slots are written.
template <int LAYOUT>
__global__ __launch_bounds__(256) void gather_record_kernel(DevVolume vol, DevParams prm,
                                                            DevCameras cams, uint32_t frame,
                                                            int W, int H, int tiles_x,
                                                            int tiles_y, int S, int L,
                                                            const uint2* __restrict__ trace,
                                                            int max_slots,
                                                            uint32_t* __restrict__ codes,
                                                            uint32_t* __restrict__ counts) {
  const int tiles_per_view = tiles_x * tiles_y;
  const int tile = xcd_walk(blockIdx.x, gridDim.x, L);
  const int view = tile / tiles_per_view;
  int tx, ty;
  supertile(tile - view * tiles_per_view, tiles_x, tiles_y, S, tx, ty);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int px, py;
  tile_pixel(tx, ty, wave, lane, px, py);
  stage_volume<LAYOUT>(vol);
  const bool inside = px < W && py < H;
  uint32_t n_prim = 0, mask = 0;
  float ox = 0.0f, oy = 0.0f, oz = 0.0f, dx = 0.0f, dy = 0.0f, dz = 1.0f, j = 0.5f;
  float tn = 0.0f, D = 0.0f;
  if (inside) {
    const uint2 tr = trace[((size_t)view * H + py) * W + px];
    const DevCamera& c = cams.c[view];
    camera_dir(c, px, py, W, H, dx, dy, dz);
    j = jitter_for(prm.jitter, (uint32_t)px, (uint32_t)py, frame, prm.seed);
    ox = c.pos[0];
    oy = c.pos[1];
    oz = c.pos[2];
    float tf;
    if (ray_box(vol, ox, oy, oz, dx, dy, dz, tn, tf)) {
      D = (tf - tn) / (float)prm.steps;
      n_prim = tr.x;
      mask = tr.y;
    }
  }
  uint32_t* out = codes + wave_index(tile, wave) * (size_t)max_slots * 64 + lane;
  int slot = 0;
  for (int i = 0; i < prm.steps; ++i) {
    const bool act = (uint32_t)i < n_prim;
    if (!__any(act)) break;
    const float t = fmaf((float)i + j, D, tn);
    const float qx = fmaf(t, dx, ox), qy = fmaf(t, dy, oy), qz = fmaf(t, dz, oz);
    out[(size_t)slot * 64] =
        act ? corner_code(vol, fmaf(qx, vol.sx, vol.ox), fmaf(qy, vol.sy, vol.oy),
                          fmaf(qz, vol.sz, vol.oz))
            : kReplaySkip;
    ++slot;
    const bool lit = act && ((mask >> i) & 1u) && prm.light_steps > 0;
    if (__any(lit)) {
      const LightPath lp = light_path<false>(vol, prm, qx, qy, qz);
      float h = 0.5f;
      for (int k = 0; k < prm.light_steps; ++k, h += 1.0f) {
        out[(size_t)slot * 64] = lit ? corner_code(vol, fmaf(h, lp.dfx, lp.fx0),
                                                   fmaf(h, lp.dfy, lp.fy0), fmaf(h, lp.dfz, lp.fz0))
                                     : kReplaySkip;
        ++slot;
      }
    }
  }
  if (lane == 0) counts[wave_index(tile, wave)] = (uint32_t)slot;
}

// Buffer loads for the replay: a lane with no lookup in a slot gets an
// offset past the end of the volume, which the hardware answers with zeros
// and no memory access, as if the lane were masked off; so a batch of slots
// needs no per-lane branch and its fetches are all in flight together.
struct ReplaySource {
  __amdgpu_buffer_rsrc_t rsrc;
  uint32_t skip;   // an offset past the end: the volume's byte size
};

__device__ __forceinline__ ReplaySource replay_source(const DevVolume& v, uint32_t bytes) {
  // word 3: the untyped-load format the gfx9 family expects
  return {__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(v.base), (short)0, (int)bytes,
                                            0x00020000),
          bytes};
}

// Byte offsets of the volume words the render's base_lookup fetches for the
// footprint with corner k (entry 0 for a dead corner), or skip offsets.
template <int DT, int LAYOUT>
struct ReplayFetch;

template <int DT>
struct ReplayFetch<DT, LAYOUT_DENSE> {
  static constexpr int kLoads = 8;
  __device__ static __forceinline__ void offsets(const DevVolume& v, int kx, int ky, int kz,
                                                 bool live, bool take, uint32_t skip,
                                                 uint32_t (&o)[kLoads]) {
    const int xb = min(kx + 1, v.nx - 1), yb = min(ky + 1, v.ny - 1), zb = min(kz + 1, v.nz - 1);
    const int ra = ky * v.row, rb = yb * v.row, pa = kz * v.plane, pb = zb * v.plane;
    const int idx[8] = {pa + ra + kx, pa + ra + xb, pa + rb + kx, pa + rb + xb,
                        pb + ra + kx, pb + ra + xb, pb + rb + kx, pb + rb + xb};
    constexpr uint32_t E = DT == DT_F32 ? 4 : 2;
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = !take ? skip : live ? (uint32_t)idx[k] * E : 0u;
  }
  __device__ static __forceinline__ uint32_t fetch(const ReplaySource& src,
                                                   const uint32_t (&o)[kLoads]) {
    uint32_t x = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if constexpr (DT == DT_F32) x ^= __builtin_amdgcn_raw_buffer_load_b32(src.rsrc, o[k], 0, 0);
      else x ^= (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(src.rsrc, o[k], 0, 0);
    }
    return x;
  }
};

template <int DT, bool TAB>
struct ReplayQuad {
  static constexpr int kLoads = 2;
  __device__ static __forceinline__ void offsets(const DevVolume& v, int kx, int ky, int kz,
                                                 bool live, bool take, uint32_t skip,
                                                 uint32_t (&o)[kLoads]) {
    entry_off_t<TAB> ia, ib;   // below 4 GiB: checked on the host
    quad_entries<TAB>(v, kx, ky, kz, ia, ib);
    o[0] = !take ? skip : live ? (uint32_t)ia : 0u;
    o[1] = !take ? skip : live ? (uint32_t)ib : 0u;
  }
  __device__ static __forceinline__ uint32_t fetch(const ReplaySource& src,
                                                   const uint32_t (&o)[kLoads]) {
    uint32_t x = 0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if constexpr (DT == DT_F32) {
        const auto q = __builtin_amdgcn_raw_buffer_load_b128(src.rsrc, o[k], 0, 0);
        x ^= q[0] ^ q[1] ^ q[2] ^ q[3];
      } else {
        const auto q = __builtin_amdgcn_raw_buffer_load_b64(src.rsrc, o[k], 0, 0);
        x ^= q[0] ^ q[1];
      }
    }
    return x;
  }
};

template <int DT, bool TAB>
struct ReplayOct {
  static constexpr int kLoads = DT == DT_F32 ? 2 : 1;
  __device__ static __forceinline__ void offsets(const DevVolume& v, int kx, int ky, int kz,
                                                 bool live, bool take, uint32_t skip,
                                                 uint32_t (&o)[kLoads]) {
    const uint32_t e = (uint32_t)packed_entry<TAB>(v, kx, ky, kz + 1);
    o[0] = !take ? skip : live ? e : 0u;
    if constexpr (kLoads == 2) o[1] = !take ? skip : o[0] + 16u;
  }
  __device__ static __forceinline__ uint32_t fetch(const ReplaySource& src,
                                                   const uint32_t (&o)[kLoads]) {
    uint32_t x = 0;
#pragma unroll
    for (int k = 0; k < kLoads; ++k) {
      const auto q = __builtin_amdgcn_raw_buffer_load_b128(src.rsrc, o[k], 0, 0);
      x ^= q[0] ^ q[1] ^ q[2] ^ q[3];
    }
    return x;
  }
};

template <int DT>
struct ReplayFetch<DT, LAYOUT_QUAD> : ReplayQuad<DT, false> {};
template <int DT>
struct ReplayFetch<DT, LAYOUT_QUAD | kLayoutTab> : ReplayQuad<DT, true> {};
template <int DT>
struct ReplayFetch<DT, LAYOUT_OCT> : ReplayOct<DT, false> {};
template <int DT>
struct ReplayFetch<DT, LAYOUT_OCT | kLayoutTab> : ReplayOct<DT, true> {};

constexpr int kReplayBatch = 8;   // slots whose fetches are in flight together

// Replays the recorded slots of every wavefront on the render's launch shape
// and tile walk (in the order of even frames; on odd ones the render takes
// each XCD's blocks in reverse), kReplayBatch slots at a time: their codes, then all their
// fetches, then the folds. RANDOM: the same slots and lanes, each at a
// uniformly random corner of the whole volume (no occupancy skip). Corners
// are clamped into the volume and slot counts to max_slots, whatever the
// buffers hold; slots past a wavefront's count are never read.
template <int DT, int LAYOUT, bool RANDOM>
__global__ __launch_bounds__(256) void gather_replay_kernel(DevVolume vol, uint32_t bytes,
                                                            int tiles, int L, int max_slots,
                                                            const uint32_t* __restrict__ codes,
                                                            const uint32_t* __restrict__ counts,
                                                            uint32_t* __restrict__ out) {
  using F = ReplayFetch<DT, LAYOUT>;
  const int tile = xcd_walk(blockIdx.x, gridDim.x, L);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  stage_volume<LAYOUT>(vol);
  if (tile >= tiles) return;
  const ReplaySource src = replay_source(vol, bytes);
  const size_t wv = wave_index(tile, wave);
  const int n = min((int)__builtin_amdgcn_readfirstlane(counts[wv]), max_slots);
  const uint32_t* in = codes + wv * (size_t)max_slots * 64 + lane;
  uint32_t acc = 0;
  for (int s0 = 0; s0 < n; s0 += kReplayBatch) {
    uint32_t c[kReplayBatch];
#pragma unroll
    for (int u = 0; u < kReplayBatch; ++u) c[u] = s0 + u < n ? in[(size_t)(s0 + u) * 64] : kReplaySkip;
    uint32_t o[kReplayBatch][F::kLoads];
#pragma unroll
    for (int u = 0; u < kReplayBatch; ++u) {
      int kx, ky, kz;
      bool live = true;
      if constexpr (RANDOM) {
        const uint32_t h = pcg((uint32_t)((wv * (size_t)max_slots + s0 + u) * 64 + lane));
        kx = (int)(((h & 0x3FFu) * (uint32_t)vol.nx) >> 10);
        ky = (int)((((h >> 10) & 0x3FFu) * (uint32_t)vol.ny) >> 10);
        kz = (int)((((h >> 20) & 0x3FFu) * (uint32_t)vol.nz) >> 10);
      } else {
        kx = min((int)(c[u] & 0x3FFu), vol.nx - 1);
        ky = min((int)((c[u] >> 10) & 0x3FFu), vol.ny - 1);
        kz = min((int)((c[u] >> 20) & 0x3FFu), vol.nz - 1);
        live = ((c[u] >> 30) & 1u) == 0u;
      }
      F::offsets(vol, kx, ky, kz, live, c[u] != kReplaySkip, src.skip, o[u]);
    }
    uint32_t x[kReplayBatch];
#pragma unroll
    for (int u = 0; u < kReplayBatch; ++u) x[u] = F::fetch(src, o[u]);
#pragma unroll
    for (int u = 0; u < kReplayBatch; ++u) acc ^= x[u];
  }
  out[wv * 64 + lane] = acc;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

template <int LAYOUT>
static hipError_t record_run(const DevVolume& v, const DevParams& p, const DevCameras& c,
                             int n_views, uint32_t frame, int W, int H, const uint32_t* trace,
                             int max_slots, uint32_t* codes, uint32_t* counts, hipStream_t s) {
  const int tiles_x = (W + 15) / 16, tiles_y = (H + 15) / 16;
  const TileWalk tw = tile_walk();
  hipLaunchKernelGGL((gather_record_kernel<LAYOUT>), dim3(tiles_x * tiles_y * n_views), dim3(256),
                     0, s, v, p, c, frame, W, H, tiles_x, tiles_y, tw.S, tw.L,
                     reinterpret_cast<const uint2*>(trace), max_slots, codes, counts);
  return hipGetLastError();
}

hipError_t launch_gather_record(const DevVolume& v, int layout, const DevParams& p,
                                const DevCameras& c, int n_views, uint32_t frame, int W, int H,
                                const uint32_t* trace, int max_slots, uint32_t* codes,
                                uint32_t* counts, hipStream_t s) {
  // the record needs the occupancy test only (entry indices are the replay's)
  switch (sampler_layout(v, layout) & 3) {
    case LAYOUT_DENSE:
      return record_run<LAYOUT_DENSE>(v, p, c, n_views, frame, W, H, trace, max_slots, codes,
                                      counts, s);
    default:
      return record_run<LAYOUT_QUAD>(v, p, c, n_views, frame, W, H, trace, max_slots, codes,
                                     counts, s);
  }
}

template <int DT, int LAYOUT, bool RANDOM>
static hipError_t replay_run(const DevVolume& v, uint32_t bytes, int tiles, int max_slots,
                             const uint32_t* codes, const uint32_t* counts, int blocks_per_cu,
                             uint32_t* out, hipStream_t s) {
  auto fn = gather_replay_kernel<DT, LAYOUT, RANDOM>;
  hipFuncAttributes attr;
  hipError_t e = hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(fn));
  if (e != hipSuccess) return e;
  const long long pad = residency_lds(blocks_per_cu, attr.sharedSizeBytes);
  if (pad < 0) return hipErrorInvalidValue;
  // the occupancy test is baked into the codes: no bitmap to stage
  DevVolume nv = v;
  nv.occ = nullptr;
  hipLaunchKernelGGL(fn, dim3(tiles), dim3(256), (size_t)pad, s, nv, bytes, tiles,
                     tile_walk().L, max_slots, codes, counts, out);
  return hipGetLastError();
}

template <int DT, int LAYOUT>
static hipError_t replay_mode(bool random, const DevVolume& v, uint32_t bytes, int tiles,
                              int max_slots, const uint32_t* codes, const uint32_t* counts,
                              int blocks_per_cu, uint32_t* out, hipStream_t s) {
  return random ? replay_run<DT, LAYOUT, true>(v, bytes, tiles, max_slots, codes, counts,
                                               blocks_per_cu, out, s)
                : replay_run<DT, LAYOUT, false>(v, bytes, tiles, max_slots, codes, counts,
                                                blocks_per_cu, out, s);
}

template <int DT>
static hipError_t replay_layout(int layout, bool random, const DevVolume& v, uint32_t bytes,
                                int tiles, int max_slots, const uint32_t* codes, const uint32_t* counts,
                                int blocks_per_cu, uint32_t* out, hipStream_t s) {
  switch (layout) {
    case LAYOUT_QUAD:
      return replay_mode<DT, LAYOUT_QUAD>(random, v, bytes, tiles, max_slots, codes, counts,
                                          blocks_per_cu, out, s);
    case LAYOUT_OCT:
      return replay_mode<DT, LAYOUT_OCT>(random, v, bytes, tiles, max_slots, codes, counts,
                                         blocks_per_cu, out, s);
    case LAYOUT_QUAD | kLayoutTab:
      return replay_mode<DT, LAYOUT_QUAD | kLayoutTab>(random, v, bytes, tiles, max_slots, codes, counts,
                                                       blocks_per_cu, out, s);
    case LAYOUT_OCT | kLayoutTab:
      return replay_mode<DT, LAYOUT_OCT | kLayoutTab>(random, v, bytes, tiles, max_slots, codes, counts,
                                                      blocks_per_cu, out, s);
    default:
      return replay_mode<DT, LAYOUT_DENSE>(random, v, bytes, tiles, max_slots, codes, counts,
                                           blocks_per_cu, out, s);
  }
}

hipError_t launch_gather_replay(const DevVolume& v, int dtype, int layout, uint32_t bytes,
                                int tiles, int max_slots, const uint32_t* codes, const uint32_t* counts,
                                bool random, int blocks_per_cu, uint32_t* out, hipStream_t s) {
  layout = sampler_layout(v, layout);
  switch (dtype) {
    case DT_F16:
      return replay_layout<DT_F16>(layout, random, v, bytes, tiles, max_slots, codes, counts,
                                   blocks_per_cu, out, s);
    case DT_BF16:
      return replay_layout<DT_BF16>(layout, random, v, bytes, tiles, max_slots, codes, counts,
                                    blocks_per_cu, out, s);
    default:
      return replay_layout<DT_F32>(layout, random, v, bytes, tiles, max_slots, codes, counts,
                                   blocks_per_cu, out, s);
  }
}

}  // namespace cloud

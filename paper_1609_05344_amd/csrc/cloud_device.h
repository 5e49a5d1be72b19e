// Device-side building blocks of the cloud raymarch (gfx950).
//
// One thread owns one ray. Nothing here uses floating-point atomics, so every
// output is bitwise reproducible. Storage types are decoded exactly to float32
// and all lerps, optical depths, exponentials and colour run in float32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "cloud_types.h"

namespace cloud {

enum { DT_F32 = 0, DT_F16 = 1, DT_BF16 = 2 };

// Light-march lookups issued back to back (independent loads in flight).
constexpr int kLightUnroll = 6;

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

// Start offset of pixel (px, py) under jitter mode m: 0 none (j = 1/2); 1 per
// pixel; 2 one offset per 8x8-pixel tile (one per wavefront); 3 one offset
// per frame. Modes 2 and 3 hash (px >> 3, py >> 3) and (0, 0) instead of
// (px, py).
__device__ __forceinline__ float jitter_for(int m, uint32_t px, uint32_t py, uint32_t frame,
                                            uint32_t seed) {
  if (m == 0) return 0.5f;
  if (m == 2) {
    px >>= 3;
    py >>= 3;
  } else if (m == 3) {
    px = 0u;
    py = 0u;
  }
  return jitter_offset(px, py, frame, seed);
}

// ---------------------------------------------------------------------------
// Texel decoding
// ---------------------------------------------------------------------------

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

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

// Two 16-bit texels packed in a word (low half first) -> two floats.
template <int DT>
__device__ __forceinline__ void unpack2(uint32_t u, float& lo, float& hi) {
  if constexpr (DT == DT_F16) {
    const half2_t h = __builtin_bit_cast(half2_t, u);
    lo = (float)h.x;
    hi = (float)h.y;
  } else {
    lo = __uint_as_float(u << 16);
    hi = __uint_as_float(u & 0xFFFF0000u);
  }
}

__device__ __forceinline__ float lerp(float a, float b, float w) { return fmaf(w, b - a, a); }

// Continuous texel coordinate bounded to [0, n - 1], split into the corner k
// and the weight w. Under clamp-to-edge a lookup is constant beyond the outer
// texel centres, and at the bound w = 0 selects the edge texel exactly, so the
// bound changes no lookup; it keeps k inside [0, n - 1] for any input (NaN
// too), which the index arithmetic below relies on.
// The clamp is one median-of-three (a NaN input gives 0); f >= 0 then, so
// the fraction is f - floor(f) exactly and truncation is the floor.
__device__ __forceinline__ void split_coord(float f, int n, float& w, int& k) {
  f = __builtin_amdgcn_fmed3f(f, 0.0f, (float)(n - 1));
  w = __builtin_amdgcn_fractf(f);
  k = (int)f;   // in [0, n - 1]
}

// ---------------------------------------------------------------------------
// Occupancy: one bit per brick, staged in LDS by every kernel that samples
// ---------------------------------------------------------------------------

static __shared__ uint32_t s_occupancy[kOccupancyWords];

// Byte-offset terms of a table-indexed packed volume (kLayoutTab): the bytes
// of entry (x + 1, y + 1, z) of packed_index are s_terms[x] +
// s_terms[kTabAxis + y] + s_terms[2 kTabAxis + z], for corners x, y and
// packed planes z; for the quad layout s_terms[3 kTabAxis + z] is the z term
// of the next plane up, min(z + 1, nz - 1), so that both planes of a lookup
// come from one table address.
static __shared__ __attribute__((aligned(16))) uint32_t s_terms[4 * kTabAxis];

__device__ __forceinline__ uint32_t packed_term(int i, int sh, int stride, int low_shift,
                                                int entry_shift) {
  return (uint32_t)((mul24(i >> sh, stride) << 3) | ((i & ((1 << sh) - 1)) << low_shift))
         << entry_shift;
}

// Byte-offset terms of a table-indexed packed layout into LDS (no barrier).
template <int LAYOUT>
__device__ __forceinline__ void build_terms(const DevVolume& v) {
  if constexpr ((LAYOUT & kLayoutTab) != 0) {
    // packed planes: 0..nz-1 (quad), 0..nz (oct); the host checked v.tab
    const int planes = (LAYOUT & 3) == LAYOUT_OCT ? v.nz + 1 : v.nz;
    const int es = v.entry_shift;
    for (int i = threadIdx.x; i < v.nx; i += blockDim.x) s_terms[i] = packed_term(i + 1, v.bx, 1, 0, es);
    for (int i = threadIdx.x; i < v.ny; i += blockDim.x)
      s_terms[kTabAxis + i] = packed_term(i + 1, v.by, v.row, v.bx, es);
    for (int i = threadIdx.x; i < planes; i += blockDim.x)
      s_terms[2 * kTabAxis + i] = packed_term(i, v.bz, v.plane, v.bx + v.by, es);
    if constexpr ((LAYOUT & 3) == LAYOUT_QUAD) {
      for (int i = threadIdx.x; i < planes; i += blockDim.x)
        s_terms[3 * kTabAxis + i] = packed_term(min(i + 1, planes - 1), v.bz, v.plane, v.bx + v.by, es);
    }
  }
}

// Copies the volume's occupancy bitmap (if any) into LDS and, for a
// table-indexed packed layout, builds the entry-index terms there. Every
// thread of the workgroup must call it before sampling (it ends with a
// barrier).
template <int LAYOUT>
__device__ __forceinline__ void stage_volume(const DevVolume& v) {
  if (v.occ) {
    for (int i = threadIdx.x; i < v.occ_words; i += blockDim.x) s_occupancy[i] = v.occ[i];
  }
  build_terms<LAYOUT>(v);
  __syncthreads();
}

// The same staging in two halves, for 256-thread workgroups: the first
// issues the bitmap loads into registers, the second stores them, builds the
// terms and waits, so that work placed between the two (a ray's set-up)
// overlaps the loads.
struct StagedOccupancy {
  uint32_t w[kOccupancyWords / 256];
};
__device__ __forceinline__ void stage_volume_begin(const DevVolume& v, StagedOccupancy& r) {
#pragma unroll
  for (int k = 0; k < kOccupancyWords / 256; ++k) {
    const int i = threadIdx.x + 256 * k;
    r.w[k] = v.occ && i < v.occ_words ? v.occ[i] : 0u;
  }
}
template <int LAYOUT>
__device__ __forceinline__ void stage_volume_end(const DevVolume& v, const StagedOccupancy& r) {
  if (v.occ) {
#pragma unroll
    for (int k = 0; k < kOccupancyWords / 256; ++k) {
      const int i = threadIdx.x + 256 * k;
      if (i < v.occ_words) s_occupancy[i] = r.w[k];
    }
  }
  build_terms<LAYOUT>(v);
  __syncthreads();
}

// False when every texel a footprint with corner k (in [0, n - 1] per axis)
// can touch is zero, so the trilinear lookup is exactly 0.
__device__ __forceinline__ bool occupied(const DevVolume& v, int kx, int ky, int kz) {
  if (!v.occ) return true;
  const int bx = kx >> v.occ_lg;
  const int by = ky >> v.occ_lg;
  const int bz = kz >> v.occ_lg;
  const int b = mul24(bz, v.occ_plane) + mul24(by, v.occ_nbx) + bx;   // < 32768
  return __builtin_amdgcn_ubfe(s_occupancy[b >> 5], (uint32_t)b, 1u) != 0u;   // bit b & 31
}

// ---------------------------------------------------------------------------
// Base-volume trilinear lookup with clamp-to-edge, x then y then z
//
// Each layout fetches the words of one footprint (load) and turns them into
// the eight texels in the order (x0,y0,z0), (x1,y0,z0), (x0,y1,z0), (x1,y1,z0),
// then the same four of plane z1 (decode). A dead lookup (empty brick) keeps
// its fetches but points them at entry 0.
// ---------------------------------------------------------------------------

template <int DT, int LAYOUT>
struct BaseSampler;

// Dense [nz][ny][nx]: eight texel fetches per lookup.
template <int DT>
struct BaseSampler<DT, LAYOUT_DENSE> {
  static constexpr int kWords = 8;
  struct Addr {
    int idx[8];
  };
  __device__ static __forceinline__ Addr addr(const DevVolume& v, int kx, int ky, int kz) {
    const int xa = kx, xb = min(kx + 1, v.nx - 1);
    const int ya = ky, yb = min(ky + 1, v.ny - 1);
    const int za = kz, zb = min(kz + 1, v.nz - 1);
    // indices stay below 2^31 and plane < 2^24 (checked on the host), so the
    // 24-bit multiplies are exact
    const int ra = __umul24(ya, v.row), rb = __umul24(yb, v.row);
    const int pa = __umul24(za, v.plane), pb = __umul24(zb, v.plane);
    const int i0 = pa + ra, i1 = pa + rb, i2 = pb + ra, i3 = pb + rb;
    return {{i0 + xa, i0 + xb, i1 + xa, i1 + xb, i2 + xa, i2 + xb, i3 + xa, i3 + xb}};
  }
  // the entry-0 redirect of a dead lookup
  __device__ static __forceinline__ Addr redirect(const Addr& a, bool live) {
    Addr r;
#pragma unroll
    for (int k = 0; k < 8; ++k) r.idx[k] = live ? a.idx[k] : 0;
    return r;
  }
  __device__ static __forceinline__ void fetch(const DevVolume& v, const Addr& a,
                                               uint32_t (&w)[kWords]) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if constexpr (DT == DT_F32) w[k] = static_cast<const uint32_t*>(v.base)[a.idx[k]];
      else w[k] = static_cast<const uint16_t*>(v.base)[a.idx[k]];
    }
  }
  __device__ static __forceinline__ void decode(const uint32_t (&w)[kWords], float (&c)[8]) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if constexpr (DT == DT_F32) c[k] = __uint_as_float(w[k]);
      else if constexpr (DT == DT_F16) c[k] = (float)__builtin_bit_cast(_Float16, (uint16_t)w[k]);
      else c[k] = __uint_as_float(w[k] << 16);
    }
  }
  // 16-bit texels as (x0, x1) pairs, low half first: rows (y0, z0), (y1, z0),
  // (y0, z1), (y1, z1).
  __device__ static __forceinline__ void pairs(const uint32_t (&w)[kWords], uint32_t (&p)[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) p[k] = w[2 * k] | (w[2 * k + 1] << 16);
  }
};

// Byte offsets into a packed volume: 32-bit with the LDS tables (the host
// admits table-indexed volumes below 4 GiB), 64-bit otherwise.
template <bool TAB>
using entry_off_t = std::conditional_t<TAB, uint32_t, uint64_t>;

// Byte offset of the entry of the footprint with corner k (kx, ky in
// [0, n - 1]) in packed plane z of a packed volume: three LDS terms (TAB) or
// the index arithmetic.
template <bool TAB>
__device__ __forceinline__ entry_off_t<TAB> packed_entry(const DevVolume& v, int kx, int ky, int z) {
  if constexpr (TAB) {
    return s_terms[kx] + s_terms[kTabAxis + ky] + s_terms[2 * kTabAxis + z];
  } else {
    return (uint64_t)(uint32_t)packed_index(kx + 1, ky + 1, z, v.bx, v.by, v.bz, v.row, v.plane)
           << v.entry_shift;
  }
}

// Byte offsets of the two entries (planes kz and min(kz + 1, nz - 1)) of a
// quad-layout lookup with corner k.
template <bool TAB>
__device__ __forceinline__ void quad_entries(const DevVolume& v, int kx, int ky, int kz,
                                             entry_off_t<TAB>& ea, entry_off_t<TAB>& eb) {
  if constexpr (TAB) {
    const uint32_t xy = s_terms[kx] + s_terms[kTabAxis + ky];
    ea = xy + s_terms[2 * kTabAxis + kz];
    eb = xy + s_terms[3 * kTabAxis + kz];
  } else {
    ea = packed_entry<false>(v, kx, ky, kz);
    eb = packed_entry<false>(v, kx, ky, min(kz + 1, v.nz - 1));
  }
}

// The word of type T (uint2 or uint4) at byte offset off of the volume. A
// table-indexed volume is below 4 GiB, so its fetches are buffer loads with
// the 32-bit offset as is (no per-lane address arithmetic); the range is the
// stored size, which every offset stays inside.
template <typename T, typename O>
__device__ __forceinline__ T volume_word(const DevVolume& v, O off) {
  if constexpr (std::is_same_v<O, uint32_t>) {
    // word 3: the untyped-load format the gfx9 family expects
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<void*>(v.base), (short)0, (int)v.tab_bytes, 0x00020000);
    if constexpr (sizeof(T) == 16) {
      const auto q = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
      return T{q[0], q[1], q[2], q[3]};
    } else {
      const auto q = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
      return T{q[0], q[1]};
    }
  } else {
    return *reinterpret_cast<const T*>(static_cast<const char*>(v.base) + off);
  }
}

// Four float32 texels, or eight 16-bit texels packed two to a word (low half
// first), to floats.
template <int DT, int N>
__device__ __forceinline__ void decode_packed(const uint32_t (&w)[N], float (&c)[8]) {
  if constexpr (DT == DT_F32) {
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = __uint_as_float(w[k]);
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) unpack2<DT>(w[k], c[2 * k], c[2 * k + 1]);
  }
}

// Quad layout, nz x (ny+1) x (nx+1) entries of 4 texels in bricks (see
// packed_index): entry (z, y, x) holds the texels at (x, y), (x+1, y),
// (x, y+1), (x+1, y+1) of plane z (edge-clamped), so a lookup is two aligned
// fetches, one per z plane.
template <int DT, bool TAB>
struct QuadSampler {
  static constexpr int kWords = DT == DT_F32 ? 8 : 4;
  struct Addr {
    entry_off_t<TAB> a, b;   // byte offsets of planes kz and kz + 1
  };
  __device__ static __forceinline__ Addr addr(const DevVolume& v, int kx, int ky, int kz) {
    entry_off_t<TAB> ia, ib;
    quad_entries<TAB>(v, kx, ky, kz, ia, ib);
    return {ia, ib};
  }
  __device__ static __forceinline__ Addr redirect(const Addr& e, bool live) {
    return {live ? e.a : 0u, live ? e.b : 0u};
  }
  __device__ static __forceinline__ void fetch(const DevVolume& v, const Addr& e,
                                               uint32_t (&w)[kWords]) {
    if constexpr (DT == DT_F32) {
      const uint4 A = volume_word<uint4>(v, e.a), B = volume_word<uint4>(v, e.b);
      w[0] = A.x; w[1] = A.y; w[2] = A.z; w[3] = A.w;
      w[4] = B.x; w[5] = B.y; w[6] = B.z; w[7] = B.w;
    } else {
      const uint2 A = volume_word<uint2>(v, e.a), B = volume_word<uint2>(v, e.b);
      w[0] = A.x; w[1] = A.y; w[2] = B.x; w[3] = B.y;
    }
  }
  __device__ static __forceinline__ void decode(const uint32_t (&w)[kWords], float (&c)[8]) {
    decode_packed<DT>(w, c);
  }
  __device__ static __forceinline__ void pairs(const uint32_t (&w)[kWords], uint32_t (&p)[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) p[k] = w[k];
  }
};

template <int DT>
struct BaseSampler<DT, LAYOUT_QUAD> : QuadSampler<DT, false> {};
template <int DT>
struct BaseSampler<DT, LAYOUT_QUAD | kLayoutTab> : QuadSampler<DT, true> {};

// Oct layout, (nz+1) x (ny+1) x (nx+1) entries of 8 texels in bricks: entry
// (z, y, x) holds the whole 2x2x2 footprint (the quad of plane z, then the
// quad of plane z+1, edge-clamped), so a lookup is one aligned fetch (two for
// float32).
template <int DT, bool TAB>
struct OctSampler {
  static constexpr int kWords = DT == DT_F32 ? 8 : 4;
  struct Addr {
    entry_off_t<TAB> e;   // byte offset of the footprint's entry
  };
  __device__ static __forceinline__ Addr addr(const DevVolume& v, int kx, int ky, int kz) {
    return {packed_entry<TAB>(v, kx, ky, kz + 1)};
  }
  __device__ static __forceinline__ Addr redirect(const Addr& a, bool live) {
    return {live ? a.e : 0u};
  }
  __device__ static __forceinline__ void fetch(const DevVolume& v, const Addr& a,
                                               uint32_t (&w)[kWords]) {
    if constexpr (DT == DT_F32) {
      const uint4 A = volume_word<uint4>(v, a.e), B = volume_word<uint4>(v, a.e + 16u);
      w[0] = A.x; w[1] = A.y; w[2] = A.z; w[3] = A.w;
      w[4] = B.x; w[5] = B.y; w[6] = B.z; w[7] = B.w;
    } else {
      const uint4 Q = volume_word<uint4>(v, a.e);
      w[0] = Q.x; w[1] = Q.y; w[2] = Q.z; w[3] = Q.w;
    }
  }
  __device__ static __forceinline__ void decode(const uint32_t (&w)[kWords], float (&c)[8]) {
    decode_packed<DT>(w, c);
  }
  __device__ static __forceinline__ void pairs(const uint32_t (&w)[kWords], uint32_t (&p)[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) p[k] = w[k];
  }
};

template <int DT>
struct BaseSampler<DT, LAYOUT_OCT> : OctSampler<DT, false> {};
template <int DT>
struct BaseSampler<DT, LAYOUT_OCT | kLayoutTab> : OctSampler<DT, true> {};

// A base-volume trilinear lookup at continuous texel coordinates f, in three
// phases: prepare (corner, weights, occupancy, entry addresses), fetch, and
// finish (the lerps).
template <int DT, int LAYOUT>
struct BaseLookup {
  using S = BaseSampler<DT, LAYOUT>;
  typename S::Addr addr;
  float wx, wy, wz;
  bool live;   // false: an empty brick, the lookup is exactly 0

  __device__ static __forceinline__ BaseLookup prepare(const DevVolume& v, float fx, float fy,
                                                       float fz) {
    BaseLookup q;
    int kx, ky, kz;
    split_coord(fx, v.nx, q.wx, kx);
    split_coord(fy, v.ny, q.wy, ky);
    split_coord(fz, v.nz, q.wz, kz);
    // the entry offsets first, so that their LDS reads (table layouts) are in
    // flight with the occupancy test's
    const typename S::Addr raw = S::addr(v, kx, ky, kz);
    q.live = occupied(v, kx, ky, kz);
    q.addr = S::redirect(raw, q.live);
    return q;
  }

  __device__ __forceinline__ void fetch(const DevVolume& v, uint32_t (&w)[S::kWords]) const {
    S::fetch(v, addr, w);
  }

  __device__ __forceinline__ float finish(const uint32_t (&w)[S::kWords]) const {
    if constexpr (DT == DT_F16) {
      // the four x-lerps as 16-bit dot products accumulated in float32:
      // a + w (b - a) = dot((a, b), (-w, w)) + a, with w rounded to half
      uint32_t p[4];
      S::pairs(w, p);
      float c[4];
      const half2_t wt = {(_Float16)(-wx), (_Float16)wx};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const half2_t h = __builtin_bit_cast(half2_t, p[k]);
        c[k] = __builtin_amdgcn_fdot2(h, wt, (float)h.x, false);
      }
      const float c0 = lerp(c[0], c[1], wy), c1 = lerp(c[2], c[3], wy);
      return live ? lerp(c0, c1, wz) : 0.0f;
    } else {
      float c[8];
      S::decode(w, c);
      const float c0 = lerp(lerp(c[0], c[1], wx), lerp(c[2], c[3], wx), wy);
      const float c1 = lerp(lerp(c[4], c[5], wx), lerp(c[6], c[7], wx), wy);
      return live ? lerp(c0, c1, wz) : 0.0f;
    }
  }
};

// Trilinear lookup of the base volume at continuous texel coordinates f. A
// lookup in an empty brick keeps its fetch, pointed at entry 0 (a line every
// wavefront shares), so that the light march's fetches stay in flight
// together, and is 0.
template <int DT, int LAYOUT>
__device__ __forceinline__ float base_lookup(const DevVolume& v, float fx, float fy, float fz) {
  const BaseLookup<DT, LAYOUT> q = BaseLookup<DT, LAYOUT>::prepare(v, fx, fy, fz);
  uint32_t w[BaseSampler<DT, LAYOUT>::kWords];
  q.fetch(v, w);
  return q.finish(w);
}

// Index k of a periodic axis of n texels, wrapped into [0, n).
__device__ __forceinline__ int wrap_index(int k, int n) {
  int r = k % n;
  return r < 0 ? r + n : r;
}

// Trilinear lookup with repeat addressing (the tiled detail volume, dense).
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

// Repeat-addressed lookup in the packed detail volume: entry (z, y, x) of
// [dnz][dny][dnx] x 8 holds the texels (x|x+1, y|y+1, z|z+1) mod n in the
// order of the oct layout, so a lookup is one aligned fetch (two for float32).
// Same lerps, in the same order, as trilerp_repeat.
template <int DT>
__device__ __forceinline__ float detail_oct(const DevVolume& v, float fx, float fy, float fz) {
  const float lim = 1048576.0f;
  fx = fminf(fmaxf(fx, -lim), lim);
  fy = fminf(fmaxf(fy, -lim), lim);
  fz = fminf(fmaxf(fz, -lim), lim);
  const float x0f = floorf(fx), y0f = floorf(fy), z0f = floorf(fz);
  const float wx = fx - x0f, wy = fy - y0f, wz = fz - z0f;
  int xa, ya, za;
  if (v.dpow2) {
    xa = (int)x0f & (v.dnx - 1);
    ya = (int)y0f & (v.dny - 1);
    za = (int)z0f & (v.dnz - 1);
  } else {
    xa = wrap_index((int)x0f, v.dnx);
    ya = wrap_index((int)y0f, v.dny);
    za = wrap_index((int)z0f, v.dnz);
  }
  const int e = (za * v.dny + ya) * v.dnx + xa;
  float a0, a1, a2, a3, b0, b1, b2, b3;
  if constexpr (DT == DT_F32) {
    const float4* q = static_cast<const float4*>(v.detail) + 2 * (size_t)e;
    const float4 A = q[0], B = q[1];
    a0 = A.x; a1 = A.y; a2 = A.z; a3 = A.w;
    b0 = B.x; b1 = B.y; b2 = B.z; b3 = B.w;
  } else {
    const uint4 Q = static_cast<const uint4*>(v.detail)[e];
    unpack2<DT>(Q.x, a0, a1);
    unpack2<DT>(Q.y, a2, a3);
    unpack2<DT>(Q.z, b0, b1);
    unpack2<DT>(Q.w, b2, b3);
  }
  const float c00 = lerp(a0, a1, wx), c10 = lerp(a2, a3, wx);
  const float c01 = lerp(b0, b1, wx), c11 = lerp(b2, b3, wx);
  return lerp(lerp(c00, c10, wy), lerp(c01, c11, wy), wz);
}

// Density at world point p (Section 1). With a detail volume the base shape
// is eroded: clamp((b - w d) / (1 - w d), 0, 1); where b <= 0 the result is 0
// whatever d is, so the detail lookup is skipped there. A packed volume keeps
// its detail packed too.
// Density from continuous texel coordinates of the base (f) and, with a
// detail volume, of the detail (g).
template <int DT, int LAYOUT, bool DETAIL>
__device__ __forceinline__ float density_tex(const DevVolume& v, float fx, float fy, float fz,
                                             float gx, float gy, float gz) {
  const float b = base_lookup<DT, LAYOUT>(v, fx, fy, fz);
  if constexpr (!DETAIL) {
    return b;
  } else {
    if (!(b > 0.0f)) return 0.0f;
    float d;
    if constexpr ((LAYOUT & 3) == LAYOUT_DENSE)
      d = trilerp_repeat<DT>(v.detail, v.dnx, v.dny, v.dnz, gx, gy, gz);
    else d = detail_oct<DT>(v, gx, gy, gz);
    const float wd = v.detail_weight * d;
    return fminf(fmaxf((b - wd) / (1.0f - wd), 0.0f), 1.0f);
  }
}

template <int DT, int LAYOUT, bool DETAIL>
__device__ __forceinline__ float density(const DevVolume& v, float px, float py, float pz) {
  if constexpr (DETAIL)
    return density_tex<DT, LAYOUT, DETAIL>(v, fmaf(px, v.sx, v.ox), fmaf(py, v.sy, v.oy),
                                           fmaf(pz, v.sz, v.oz), fmaf(px, v.dsx, v.dox),
                                           fmaf(py, v.dsy, v.doy), fmaf(pz, v.dsz, v.doz));
  else
    return density_tex<DT, LAYOUT, DETAIL>(v, fmaf(px, v.sx, v.ox), fmaf(py, v.sy, v.oy),
                                           fmaf(pz, v.sz, v.oz), 0.0f, 0.0f, 0.0f);
}

// Sample points of the light march from p (Section 1): L midpoints of equal
// steps up to the box exit along s, as continuous texel coordinates of the
// base (f0 + h df) and of the detail (g0 + h dg), h = k + 1/2, and the step
// length dl. The map from world to texel coordinates is affine, so the points
// are stepped in texel coordinates directly.
struct LightPath {
  float fx0, fy0, fz0, dfx, dfy, dfz;
  float gx0, gy0, gz0, dgx, dgy, dgz;
  float dl;
};

template <bool DETAIL>
__device__ __forceinline__ LightPath light_path(const DevVolume& v, const DevParams& P, float px,
                                                float py, float pz) {
  float tx = 3.402823466e38f;
  if (P.s_axis[0]) tx = fminf(tx, (P.light_bound[0] - px) * P.inv_s[0]);
  if (P.s_axis[1]) tx = fminf(tx, (P.light_bound[1] - py) * P.inv_s[1]);
  if (P.s_axis[2]) tx = fminf(tx, (P.light_bound[2] - pz) * P.inv_s[2]);
  LightPath lp;
  lp.dl = tx * P.inv_light_steps;
  const float stx = lp.dl * P.s[0], sty = lp.dl * P.s[1], stz = lp.dl * P.s[2];
  lp.fx0 = fmaf(px, v.sx, v.ox);
  lp.fy0 = fmaf(py, v.sy, v.oy);
  lp.fz0 = fmaf(pz, v.sz, v.oz);
  lp.dfx = stx * v.sx;
  lp.dfy = sty * v.sy;
  lp.dfz = stz * v.sz;
  lp.gx0 = lp.gy0 = lp.gz0 = lp.dgx = lp.dgy = lp.dgz = 0.0f;
  if constexpr (DETAIL) {
    lp.gx0 = fmaf(px, v.dsx, v.dox);
    lp.gy0 = fmaf(py, v.dsy, v.doy);
    lp.gz0 = fmaf(pz, v.dsz, v.doz);
    lp.dgx = stx * v.dsx;
    lp.dgy = sty * v.dsy;
    lp.dgz = stz * v.dsz;
  }
  return lp;
}

// Transmittance towards the sun from p (Section 1): Beer-Lambert over the
// sum of the light-march samples.
template <int DT, int LAYOUT, bool DETAIL>
__device__ __forceinline__ float light_transmittance(const DevVolume& v, const DevParams& P,
                                                     float px, float py, float pz) {
  const LightPath lp = light_path<DETAIL>(v, P, px, py, pz);
  float acc = 0.0f, h = 0.5f;   // h = k + 1/2, exact in float32
#pragma unroll kLightUnroll
  for (int k = 0; k < P.light_steps; ++k, h += 1.0f) {
    acc += density_tex<DT, LAYOUT, DETAIL>(v, fmaf(h, lp.dfx, lp.fx0), fmaf(h, lp.dfy, lp.fy0),
                                           fmaf(h, lp.dfz, lp.fz0), fmaf(h, lp.dgx, lp.gx0),
                                           fmaf(h, lp.dgy, lp.gy0), fmaf(h, lp.dgz, lp.gz0));
  }
  return exp2f(-P.alpha_log2e * lp.dl * acc);
}

// Entry and exit distances of the ray (o, d) through the volume's box (slab
// test); an axis with d_k == 0 passes iff the origin lies in its slab. False
// when the ray misses.
__device__ __forceinline__ bool ray_box(const DevVolume& v, float ox, float oy, float oz, float dx,
                                        float dy, float dz, float& tn, float& tf) {
  tn = 0.0f;
  tf = 3.402823466e38f;
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
  return hit && tf > tn;
}

struct RayResult {
  float r, g, b, a;
  // counted only on request: density lookups performed, primary samples
  // taken (up to the early exit), and bit i set when sample i (i < 32) ran a
  // light march
  uint32_t lookups, primary, light_mask;
  // on request: the ray's representative depth -- the mean sample distance
  // weighted by the opacity each step adds, where alpha >= kDepthAlphaMin;
  // the middle of the ray's chord through the box below that; 0 (at
  // infinity) when the ray misses the box
  float depth;
};

constexpr float kDepthAlphaMin = 0.01f;

// One primary ray through the volume (Sections 1, 3.1, 3.2). (o, d): origin
// and unit direction; j: start offset in [0, 1).
template <int DT, int LAYOUT, bool DETAIL, bool COUNT, bool DEPTH = false>
__device__ __forceinline__ RayResult march(const DevVolume& v, const DevParams& P, float ox,
                                           float oy, float oz, float dx, float dy, float dz,
                                           float j) {
  RayResult res = {0.0f, 0.0f, 0.0f, 0.0f, 0u, 0u, 0u, 0.0f};
  float tn, tf;
  if (!ray_box(v, ox, oy, oz, dx, dy, dz, tn, tf)) return res;

  const float D = (tf - tn) / (float)P.steps;
  const float mu = dx * P.s[0] + dy * P.s[1] + dz * P.s[2];
  const float q = fmaf(-P.hg_b, mu, P.hg_a);
  const float phase = P.hg_k / (q * sqrtf(q));
  const float sr = P.sun[0] * phase, sg = P.sun[1] * phase, sb = P.sun[2] * phase;
  const float kx = P.alpha_log2e * D;   // exp2 scale of rho for one step
  const float xD = P.alpha * D;         // optical depth per unit density for one step

  float T = 1.0f, Sr = 0.0f, Sg = 0.0f, Sb = 0.0f;
  float td = 0.0f;   // sum of (opacity added) x (sample distance), for DEPTH
  uint32_t n = 0, prim = 0, mask = 0;
  for (int i = 0; i < P.steps; ++i) {
    const float t = fmaf((float)i + j, D, tn);
    const float px = fmaf(t, dx, ox), py = fmaf(t, dy, oy), pz = fmaf(t, dz, oz);
    const float rho = density<DT, LAYOUT, DETAIL>(v, px, py, pz);
    if constexpr (COUNT) {
      n += 1;
      prim += 1;
    }
    if (rho > 0.0f) {
      float TL = 1.0f;
      if (P.light_steps > 0) {
        TL = light_transmittance<DT, LAYOUT, DETAIL>(v, P, px, py, pz);
        if constexpr (COUNT) {
          n += (uint32_t)P.light_steps;
          if (i < 32) mask |= 1u << i;
        }
      }
      const float lr = fmaf(sr, TL, P.amb[0]), lg = fmaf(sg, TL, P.amb[1]),
                  lb = fmaf(sb, TL, P.amb[2]);
      const float e = exp2f(-rho * kx);
      const float T_before = T;
      float w;
      if (P.integration) {
        // Section 3.1: T0 L_in (1 - e^{-rho alpha D}), then the T update
        w = T * (1.0f - e);
        T *= e;
      } else {
        // the basic rule: update T first, then S += T rho alpha D L_in
        T *= e;
        w = T * (rho * xD);
      }
      Sr = fmaf(w, lr, Sr);
      Sg = fmaf(w, lg, Sg);
      Sb = fmaf(w, lb, Sb);
      if constexpr (DEPTH) td = fmaf(T_before - T, t, td);
      if (T < P.t_eps) break;
    }
  }
  res.r = Sr;
  res.g = Sg;
  res.b = Sb;
  res.a = 1.0f - T;
  if constexpr (DEPTH) res.depth = res.a >= kDepthAlphaMin ? td / res.a : 0.5f * (tn + tf);
  res.lookups = n;
  res.primary = prim;
  res.light_mask = mask;
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

// Pixel of a lane in a 16x16 render tile (tx, ty): the four wavefronts of
// the workgroup each cover an 8x8 patch, so the 64 rays of a wavefront are a
// compact bundle.
__device__ __forceinline__ void tile_pixel(int tx, int ty, int wave, int lane, int& px, int& py) {
  px = tx * 16 + (wave & 1) * 8 + (lane & 7);
  py = ty * 16 + (wave >> 1) * 8 + (lane >> 3);
}

// Block index b of nb -> position in the tile walk. Workgroups are dealt to
// the 8 XCDs round-robin (b % 8 names the XCD, and each XCD has its own L2).
// The walk is cut into rounds of 8 runs of L consecutive tiles; in round j,
// XCD x takes run (x + 3j) mod 8. With L = S * S a run is one super-tile, so
// the tiles an XCD works on together still share its L2, while its runs are
// spread over the whole image: the XCDs get near-equal shares of the costly
// tiles (with one contiguous run each, the XCD holding the densest band of
// cloud would finish last). The tail that fills no round, or the whole walk
// when L == 0, is cut into 8 contiguous runs. The map is a bijection on
// [0, nb).
__device__ __forceinline__ int xcd_walk(int b, int nb, int L) {
  const int x = b & 7;
  int k = b >> 3, base = 0, n = nb;
  if (L > 0) {
    const int J = nb / (8 * L);   // full rounds
    if (k < J * L) {
      const int j = k / L;
      return (j * 8 + ((x + 3 * j) & 7)) * L + (k - j * L);
    }
    base = 8 * L * J;
    n = nb - base;
    k -= J * L;
  }
  const int q = n >> 3, r = n & 7;
  return base + x * q + min(x, r) + k;
}

// Ordered tile index k of one view -> tile (tx, ty). Tiles are walked in
// super-tiles of S x S tiles (super-tile rows top to bottom, super-tiles left
// to right, tiles row-major inside; edge super-tiles are narrower/shorter), so
// that a contiguous run of k -- what one XCD works on at a time -- covers a
// compact patch of the image, whose rays read a compact part of the volume.
// S == 0 walks the tiles row-major. The map is a bijection on [0, tx * ty).
__device__ __forceinline__ void supertile(int k, int tiles_x, int tiles_y, int S, int& tx,
                                          int& ty) {
  if (S <= 0) {
    ty = k / tiles_x;
    tx = k - ty * tiles_x;
    return;
  }
  const int band = S * tiles_x;                 // tiles in a full super-tile row
  const int R = min(k / band, (tiles_y - 1) / S);
  const int h = min(S, tiles_y - R * S);        // height of this super-tile row
  const int o = k - R * band;
  const int C = o / (S * h);
  const int w = min(S, tiles_x - C * S);
  const int l = o - C * S * h;
  const int lr = l / w;
  ty = R * S + lr;
  tx = C * S + (l - lr * w);
}

// Sum of a 32-bit value over the wavefront (all 64 lanes must be active).
__device__ __forceinline__ uint32_t wave_sum(uint32_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

}  // namespace cloud

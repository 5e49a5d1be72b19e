// Host-side launchers of the kernels (argument checks happen before these).
#pragma once

#include <hip/hip_runtime.h>

#include "cloud_types.h"

namespace cloud {

// Launch-shape knobs (process-wide; set through cloud_tune).
struct Tuning {
  // render tile walk: S x S super-tiles (0 = row-major; -1 = 4)
  int supertile = -1;
  // tiles per XCD run: the walk is dealt to the XCDs in rounds of runs this
  // long (0: one contiguous eighth per XCD; -1 = S * S, one super-tile)
  int xcd_run = -1;
  int taa_tile = 32;   // resolve tile width in pixels (16, 32 or 64; 256 pixels a tile)
  // cap on resident render workgroups per CU (0: none, the default; with the
  // bricked packed layouts every measured cap was slower)
  int render_blocks_per_cu = 0;
  // cap on the persistent serving render's workgroups per CU, read when a
  // server is created (0: automatic, by the stored volume's size)
  int serve_blocks_per_cu = 0;
};
Tuning& tuning();

// Layout argument of the sampling kernels for a volume: a packed layout whose
// volume fits the LDS byte-offset tables (DevVolume::tab) carries kLayoutTab.
inline int sampler_layout(const DevVolume& v, int layout) {
  return layout != LAYOUT_DENSE && v.tab ? layout | kLayoutTab : layout;
}

// Render tile walk under the current
// tuning: super-tile side S and XCD run length L (0 = contiguous runs).
struct TileWalk {
  int S, L;
};
TileWalk tile_walk();

// Dynamic LDS bytes that cap a 256-thread kernel using static_lds bytes of
// LDS at blocks_per_cu resident workgroups per CU on the current device (0
// when blocks_per_cu <= 0; -1 when the cap cannot be reached this way).
long long residency_lds(int blocks_per_cu, size_t static_lds);


// Render n_views (<= kMaxViews) cameras into out [n_views][H][W][4]. With
// counts or trace given, store no image: add the density lookups to *counts
// and/or write each pixel's (primary samples, light-march mask) to trace
// [n_views][H][W][2]. With depth given, also store each pixel's
// representative depth in depth [n_views][H][W].
hipError_t launch_render(const DevVolume& v, int dtype, int layout, const DevParams& p,
                         const DevCameras& c, int n_views, uint32_t frame, int W, int H,
                         float* out, unsigned long long* counts, uint32_t* trace,
                         float* depth, hipStream_t s);

// Up-sample the lw x lh layer to W x H and composite it over bg into out.
hipError_t launch_composite(const float* layer, int lw, int lh, const float* bg, float* out, int W,
                            int H, hipStream_t s);

// Temporal resolve with camera reprojection (out must not alias hist).
hipError_t launch_taa_reproject(const float* cur, const float* depth, const float* hist,
                                float* out, const DevCamera& cam, const DevCamera& prev, int W,
                                int H, float blend, hipStream_t s);

// Fetch-only replay of a render's lookups (random == false: the positions
// recorded in trace; random == true: as many lookups per pixel at uniformly
// random footprints of the volume) into out [n_views][H][W][4].
// Record the render's lookups of n_views (<= kMaxViews) views as corner
// codes per wavefront slot, and replay recorded codes (see gather.hip).
hipError_t launch_gather_record(const DevVolume& v, int layout, const DevParams& p,
                                const DevCameras& c, int n_views, uint32_t frame, int W, int H,
                                const uint32_t* trace, int max_slots, uint32_t* codes,
                                uint32_t* counts, hipStream_t s);
hipError_t launch_gather_replay(const DevVolume& v, int dtype, int layout, uint32_t bytes,
                                int tiles, int max_slots, const uint32_t* codes, const uint32_t* counts,
                                bool random, int blocks_per_cu, uint32_t* out, hipStream_t s);

// March n explicit rays into out [n][4].
hipError_t launch_rays(const DevVolume& v, int dtype, int layout, const DevParams& p,
                       uint32_t frame, const float* o, const float* d, const uint32_t* pxy,
                       long long n, float* out, hipStream_t s);

// Pack a dense [nz][ny][nx] volume of 2- or 4-byte texels into a quad or oct
// layout at dst, entries in bricks of brick[0..2] (log2 per axis).
hipError_t launch_pack(const void* src, int elem_bytes, int nx, int ny, int nz, int layout,
                       const int* brick, void* dst, hipStream_t s);

// Pack a dense repeat-addressed detail volume into its oct-wrap layout.
hipError_t launch_pack_detail(const void* src, int elem_bytes, int nx, int ny, int nz, void* dst,
                              hipStream_t s);

// Build the occupancy bitmap (nbx * nby * nbz bricks of 2^lg texels) of a
// dense volume of 2- or 4-byte texels into out.
hipError_t launch_occupancy(const void* src, int elem_bytes, int nx, int ny, int nz, int lg,
                            int nbx, int nby, int nbz, uint32_t* out, hipStream_t s);

// Jitter offsets (as integers j * 2^24) of n pixels.
hipError_t launch_jitter(const uint32_t* pxy, long long n, uint32_t frame, uint32_t seed,
                         uint32_t* out, hipStream_t s);

// Temporal resolve, or a plain copy of cur when copy is set.
hipError_t launch_taa(const float* cur, const float* hist, float* out, int W, int H, float blend,
                      bool copy, hipStream_t s);

// Whether the resolve of a W x H frame deals each XCD one contiguous run of
// its tiles.
int taa_xcd_runs(int W, int H);

// One launch: the render of n_views (<= kMaxViews) views (frame, into out)
// and the resolve of the previous frame's (prev against hist into resolved,
// or a copy of prev when copy is set), all [n_views][H][W][4].
hipError_t launch_render_resolve(const DevVolume& v, int dtype, int layout, const DevParams& p,
                                 const DevCameras& c, int n_views, uint32_t frame, int W, int H,
                                 float* out, const float* prev, const float* hist,
                                 float* resolved, float blend, bool copy, hipStream_t s);

}  // namespace cloud

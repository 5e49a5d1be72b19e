// Device descriptor table of one serving batch (host and device view).
//
// The host fills a pinned copy per batch slot; the captured graph copies it
// to the device and runs the persistent render kernel and the batched resolve
// over every request in it. The work counters sit in the table, so the
// per-batch copy also resets them (no memset node in the graph).
#pragma once

#include <stdint.h>

#include "cloud_types.h"

namespace cloud {

constexpr int kMaxBatch = 64;   // requests per batch
constexpr int kServeTaaW = 32, kServeTaaH = 8;   // resolve tile (256 pixels, full-line rows)

struct ServeItem {
  DevCamera cam;
  DevParams prm;
  int width, height;
  int tiles_x, tiles_y;
  int tile_begin;               // first global render tile (16 x 16) of this request
  int reset;                    // 1: no usable history, the frame is copied
  uint32_t frame;
  int taa_tiles_x;              // resolve tiles (kServeTaaW x kServeTaaH) per row
  int taa_tile_begin;           // first global resolve tile of this request
  int pad[3];
  void* cur;                    // [H][W] float4 scratch: this frame before resolve
  const void* hist_in;          // [H][W] float4 history read by the resolve
  void* hist_out;               // [H][W] float4 history kept by the library (or null)
  void* out;                    // [H][W] float4 caller output
};

// The per-XCD work counters sit 256 bytes apart: device-wide atomics on one
// line are serialised, and with all eight in one line the counters alone
// throttled the render (measured: 5-7 % more served frames/s apart).
constexpr int kCounterStride = 64;

struct ServeTable {
  unsigned int counters[8 * kCounterStride];   // per-XCD render work counters
  int total_tiles;
  int total_taa_tiles;
  int n_items;
  float blend;
  int supertile;
  int xcd_run;                  // tiles per XCD run of the render's walk (xcd_walk)
  ServeItem items[kMaxBatch];
};

}  // namespace cloud

// Serving: persistent batched render + resolve kernels, the HIP executor
// behind the scheduler, and the cloud_serve_* C ABI.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/cloud.h"
#include "cloud_device.h"
#include "cloud_launch.h"
#include "cloud_prepare.h"
#include "serve_core.h"
#include "serve_types.h"
#include "stream_io.h"

namespace cloud {

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Image pointers come out of the request table as generic pointers; they
// always address device global memory, so they are used as such (global
// rather than flat memory instructions).
// (The host pass of the compiler only type-checks kernel bodies; it keeps the
// generic type.)
#if defined(__HIP_DEVICE_COMPILE__)
typedef __attribute__((address_space(1))) float4 global_float4;
#else
typedef float4 global_float4;
#endif
__device__ __forceinline__ global_float4* as_global(void* p) { return (global_float4*)p; }

// Index of the request owning global tile t (requests are in tile order);
// RESOLVE selects the resolve tiling instead of the render tiling.
template <bool RESOLVE = false>
__device__ __forceinline__ int find_item(const ServeTable* tab, int n_items, int t) {
  int lo = 0, hi = n_items - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int begin = RESOLVE ? tab->items[mid].taa_tile_begin : tab->items[mid].tile_begin;
    if (begin <= t) lo = mid;
    else hi = mid - 1;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

// Persistent render over every tile of every request in the batch. The
// batch's tiles (requests back to back, each in super-tile order) are walked
// as the plain render walks one launch's tiles: block b of the walk covers
// tile xcd_walk(b), and the dispatcher would hand block b to XCD b % 8. Here
// the workgroups of XCD x (blockIdx % 8 names the XCD a workgroup most likely
// runs on) take the blocks b = x, x + 8, x + 16, ... in order from the XCD's
// own counter, so each XCD covers the same tiles, in the same order, as in a
// plain launch: compact runs that share its L2, spread over the batch for
// balance. A workgroup whose sequence is empty helps the other XCDs'; every
// workgroup leaves once all eight are empty.
// The table is read-only here apart from its work counters, which come in as
// their own pointer: with the table const and unaliased, the request fields
// are scalar loads held in scalar registers rather than per-lane copies.
template <int DT, int LAYOUT, bool DETAIL>
__global__ __launch_bounds__(256) void serve_render_kernel(DevVolume vol,
                                                           unsigned int* __restrict__ counters,
                                                           const ServeTable* __restrict__ tab) {
  stage_volume<LAYOUT>(vol);
  __shared__ int s_block;
  const int total = tab->total_tiles, n_items = tab->n_items, S = tab->supertile;
  const int L = tab->xcd_run;
  const int home = blockIdx.x & 7;
  for (int probe = 0; probe < 8;) {
    const int q = (home + probe) & 7;
    const int n_q = (total - q + 7) >> 3;   // blocks b < total with b % 8 == q
    if (threadIdx.x == 0) s_block = (int)atomicAdd(&counters[q * kCounterStride], 1u);
    __syncthreads();
    const int k = __builtin_amdgcn_readfirstlane(s_block);
    __syncthreads();
    if (k >= n_q) {
      ++probe;
      continue;
    }
    const int t = xcd_walk(8 * k + q, total, L);
    const int i = find_item(tab, n_items, t);
    const ServeItem& it = tab->items[i];
    int tx, ty;
    supertile(t - it.tile_begin, it.tiles_x, it.tiles_y, S, tx, ty);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int px, py;
    tile_pixel(tx, ty, wave, lane, px, py);
    if (px < it.width && py < it.height) {
      float dx, dy, dz;
      camera_dir(it.cam, px, py, it.width, it.height, dx, dy, dz);
      const float j =
          jitter_for(it.prm.jitter, (uint32_t)px, (uint32_t)py, it.frame, it.prm.seed);
      const RayResult r = march<DT, LAYOUT, DETAIL, false>(vol, it.prm, it.cam.pos[0],
                                                           it.cam.pos[1], it.cam.pos[2], dx, dy,
                                                           dz, j);
      // streamed: the batch's frames are resolved only after all of them
      // are rendered, from memory, so caching them would only evict volume
      store_stream(as_global(it.cur) + (size_t)py * it.width + px,
                   make_float4(r.r, r.g, r.b, r.a));
    }
  }
}

// Batched temporal resolve: every resolve tile (32 x 8 pixels, rows of whole
// 128-byte lines) of every request, grid-strided. A request without usable
// history copies its frame; otherwise the 3x3 neighbourhood clamp and blend
// of the single-frame resolve, the tile and its one-pixel halo staged in LDS.
// The result goes to the caller's output and, where the library keeps the
// stream's history, to that history too. The history read may be the output
// itself (a stream that reuses one output buffer): each pixel's history is
// read and written by the same thread.
__global__ __launch_bounds__(256) void serve_taa_kernel(const ServeTable* __restrict__ tab) {
  constexpr int TW = kServeTaaW, TH = kServeTaaH;
  __shared__ float4 tile[TH + 2][TW + 2];
  const int total = tab->total_taa_tiles, n_items = tab->n_items;
  const float blend = tab->blend;
  const int lx = threadIdx.x % TW, ly = threadIdx.x / TW;
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    const int i = find_item<true>(tab, n_items, t);
    const ServeItem& it = tab->items[i];
    const int W = it.width, H = it.height;
    const int k = t - it.taa_tile_begin;
    const int tyi = k / it.taa_tiles_x, txi = k - tyi * it.taa_tiles_x;
    const int bx = txi * TW, by = tyi * TH;
    const global_float4* cur = as_global(it.cur);
    const global_float4* hist_in = as_global(const_cast<void*>(it.hist_in));
    global_float4* hist_out = as_global(it.hist_out);
    global_float4* out = as_global(it.out);
    const int px = bx + lx, py = by + ly;
    const bool inside = px < W && py < H;
    const size_t p = (size_t)py * W + px;
    if (it.reset) {
      if (inside) {
        const float4 v = cur[p];
        if (hist_out) store_stream(hist_out + p, v);
        store_stream(out + p, v);
      }
      continue;
    }
    for (int e = threadIdx.x; e < (TH + 2) * (TW + 2); e += 256) {
      const int ey = e / (TW + 2), ex = e - ey * (TW + 2);
      const int gx = min(max(bx + ex - 1, 0), W - 1);
      const int gy = min(max(by + ey - 1, 0), H - 1);
      tile[ey][ex] = cur[(size_t)gy * W + gx];
    }
    __syncthreads();
    if (inside) {
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
      float4 h = load_stream(hist_in + p);
      h.x = fminf(fmaxf(h.x, lo.x), hi.x);
      h.y = fminf(fmaxf(h.y, lo.y), hi.y);
      h.z = fminf(fmaxf(h.z, lo.z), hi.z);
      h.w = fminf(fmaxf(h.w, lo.w), hi.w);
      const float4 r = make_float4(fmaf(blend, c.x - h.x, h.x), fmaf(blend, c.y - h.y, h.y),
                                   fmaf(blend, c.z - h.z, h.z), fmaf(blend, c.w - h.w, h.w));
      if (hist_out) store_stream(hist_out + p, r);
      store_stream(out + p, r);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// HIP executor
// ---------------------------------------------------------------------------

namespace {

struct Payload {
  DevCamera cam;
  DevParams prm;
};

typedef void (*RenderFn)(DevVolume, unsigned int*, const ServeTable*);

template <int DT, int LAYOUT>
RenderFn pick_l(bool detail) {
  return detail ? serve_render_kernel<DT, LAYOUT, true> : serve_render_kernel<DT, LAYOUT, false>;
}

template <int DT>
RenderFn pick_dt(int layout, bool detail) {
  switch (layout) {
    case LAYOUT_QUAD: return pick_l<DT, LAYOUT_QUAD>(detail);
    case LAYOUT_OCT: return pick_l<DT, LAYOUT_OCT>(detail);
    case LAYOUT_QUAD | kLayoutTab: return pick_l<DT, LAYOUT_QUAD | kLayoutTab>(detail);
    case LAYOUT_OCT | kLayoutTab: return pick_l<DT, LAYOUT_OCT | kLayoutTab>(detail);
    default: return pick_l<DT, LAYOUT_DENSE>(detail);
  }
}

RenderFn pick(int dtype, int layout, bool detail) {
  switch (dtype) {
    case DT_F16: return pick_dt<DT_F16>(layout, detail);
    case DT_BF16: return pick_dt<DT_BF16>(layout, detail);
    default: return pick_dt<DT_F32>(layout, detail);
  }
}

constexpr int kSlots = 2;
// Batch start lead: enough for the table copy and graph launch to be queued
// before the work ahead ends (the scheduler adds an eighth of that work).
constexpr int kDefaultStartLeadUs = 300;
// Over a stored volume several times the 256 MB last-level cache, fewer rays
// in flight miss less, and the persistent render holds 4 workgroups a CU
// (measured, served FP16 quad: a 1.07 GB volume 3-4 % faster at 1080p and 4K
// streams; a 134 MB one 6-7 % slower, a 268 MB one within 2 %).
constexpr size_t kLargeVolumeBytes = size_t(512) << 20;
constexpr int kLargeVolumeBlocksPerCu = 4;

// Batches run on one queue (queues = 1): table copy, persistent render and
// batched resolve in order. With two queues the resolves run on the second:
// a batch's resolve (memory-bound) waits for its render and for the previous
// resolve, and overlaps the next batch's render (bound by the vector ALUs and
// the texture path). A stream's consecutive requests may then be rendered
// while the previous one is still being resolved, so each stream has two
// scratch frames, used alternately.
class HipExecutor : public serve::Executor {
 public:
  HipExecutor(int device, const DevVolume& v, size_t volume_bytes, int dtype, int layout,
              float blend, bool graphs, int queues, bool history_in_output)
      : device_(device), vol_(v), volume_bytes_(volume_bytes), blend_(blend), graphs_(graphs),
        split_(queues == 2), history_in_output_(history_in_output) {
    fn_ = pick(dtype, sampler_layout(v, layout), v.detail != nullptr);
  }

  int init(std::string* msg) {
    hipError_t e = hipSetDevice(device_);
    if (e != hipSuccess) return err(e, msg);
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device_);
    if (e != hipSuccess) return err(e, msg);
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(fn_),
                                                     256, 0);
    if (e != hipSuccess || per_cu < 1) per_cu = 4;
    const int cap = tuning().serve_blocks_per_cu;
    if (cap > 0) per_cu = std::min(per_cu, cap);
    else if (volume_bytes_ > kLargeVolumeBytes) per_cu = std::min(per_cu, kLargeVolumeBlocksPerCu);
    render_blocks_ = cus * per_cu;
    taa_blocks_ = cus * 8;
    for (int q = 0; q < (split_ ? 2 : 1); ++q)
      if ((e = hipStreamCreateWithFlags(&stream_[q], hipStreamNonBlocking)) != hipSuccess) return err(e, msg);
    for (int s = 0; s < kSlots; ++s) {
      if ((e = hipEventCreateWithFlags(&event_[s], hipEventDisableTiming)) != hipSuccess) return err(e, msg);
      if (split_ && (e = hipEventCreateWithFlags(&rendered_[s], hipEventDisableTiming)) != hipSuccess)
        return err(e, msg);
      if ((e = hipHostMalloc(reinterpret_cast<void**>(&host_[s]), sizeof(ServeTable), hipHostMallocDefault)) != hipSuccess)
        return err(e, msg);
      std::memset(host_[s], 0, sizeof(ServeTable));
      if ((e = hipMalloc(reinterpret_cast<void**>(&dev_[s]), sizeof(ServeTable))) != hipSuccess)
        return err(e, msg);
      if (graphs_ && (e = capture(s)) != hipSuccess) return err(e, msg);
    }
    return CLOUD_OK;
  }

  ~HipExecutor() override {
    (void)hipSetDevice(device_);
    for (int q = 0; q < 2; ++q)
      if (stream_[q]) (void)hipStreamSynchronize(stream_[q]);
    for (int s = 0; s < kSlots; ++s) {
      for (int g = 0; g < 2; ++g) {
        if (exec_[s][g]) (void)hipGraphExecDestroy(exec_[s][g]);
        if (graph_[s][g]) (void)hipGraphDestroy(graph_[s][g]);
      }
      if (dev_[s]) (void)hipFree(dev_[s]);
      if (host_[s]) (void)hipHostFree(host_[s]);
      if (event_[s]) (void)hipEventDestroy(event_[s]);
      if (rendered_[s]) (void)hipEventDestroy(rendered_[s]);
    }
    for (int q = 0; q < 2; ++q)
      if (stream_[q]) (void)hipStreamDestroy(stream_[q]);
  }

  void thread_init() override { (void)hipSetDevice(device_); }

  // Scratch frames (two with a resolve queue), plus the history unless it
  // lives in the outputs.
  size_t stream_bytes(int w, int h) override {
    return (scratch_frames() + (history_in_output_ ? 0 : 1)) * frame_bytes(w, h);
  }

  // Device time of a request is roughly its samples: a primary step plus,
  // where there is cloud, the light march's steps; the resolve is a few
  // samples' worth a pixel.
  double cost(const serve::Item& r) override {
    Payload pl;
    std::memcpy(&pl, r.payload.data(), sizeof pl);
    return (double)r.width * r.height * (pl.prm.steps * (1.0 + 0.5 * pl.prm.light_steps) + 4.0);
  }

  int alloc(size_t bytes, void** mem) override {
    return hipMalloc(mem, bytes) == hipSuccess ? 0 : CLOUD_E_NOMEM;
  }

  void release(void* mem) override { (void)hipFree(mem); }

  int launch(int slot, const std::vector<serve::Item>& items) override {
    ServeTable* t = host_[slot];
    int tile = 0, taa_tile = 0;
    for (size_t i = 0; i < items.size(); ++i) {
      const serve::Item& r = items[i];
      ServeItem& it = t->items[i];
      Payload pl;
      std::memcpy(&pl, r.payload.data(), sizeof pl);
      it.cam = pl.cam;
      it.prm = pl.prm;
      it.width = r.width;
      it.height = r.height;
      it.tiles_x = (r.width + 15) / 16;
      it.tiles_y = (r.height + 15) / 16;
      it.tile_begin = tile;
      it.taa_tiles_x = (r.width + kServeTaaW - 1) / kServeTaaW;
      it.taa_tile_begin = taa_tile;
      taa_tile += it.taa_tiles_x * ((r.height + kServeTaaH - 1) / kServeTaaH);
      it.reset = r.reset_history ? 1 : 0;
      it.frame = r.frame;
      char* mem = static_cast<char*>(r.stream_mem);
      const size_t fb = frame_bytes(r.width, r.height);
      it.cur = mem + (scratch_frames() == 2 ? (r.seq & 1) * fb : 0);
      if (history_in_output_) {
        // the history is the previous request's output
        it.hist_in = r.reset_history ? nullptr : r.prev_out;
        it.hist_out = nullptr;
      } else {
        it.hist_out = mem + scratch_frames() * fb;
        it.hist_in = it.hist_out;
      }
      it.out = r.out;
      tile += it.tiles_x * it.tiles_y;
    }
    std::memset(t->counters, 0, sizeof t->counters);
    t->total_tiles = tile;
    t->total_taa_tiles = taa_tile;
    t->n_items = (int)items.size();
    t->blend = blend_;
    const TileWalk tw = tile_walk();
    t->supertile = tw.S;
    t->xcd_run = tw.L;
    hipError_t e = graphs_ ? hipGraphLaunch(exec_[slot][0], stream_[0]) : enqueue_render(slot);
    if (split_) {
      // the resolve waits for this render (and, on its queue, for the
      // previous resolve)
      if (e == hipSuccess) e = hipEventRecord(rendered_[slot], stream_[0]);
      if (e == hipSuccess) e = hipStreamWaitEvent(stream_[1], rendered_[slot], 0);
      if (e == hipSuccess)
        e = graphs_ ? hipGraphLaunch(exec_[slot][1], stream_[1]) : enqueue_resolve(slot);
    }
    if (e == hipSuccess) e = hipEventRecord(event_[slot], stream_[split_ ? 1 : 0]);
    if (e != hipSuccess) return CLOUD_E_HIP;
    // a trace range per batch, from its launch to the moment it is seen done
    char name[48];
    std::snprintf(name, sizeof name, "serve batch: %d requests", (int)items.size());
    range_[slot] = roctxRangeStartA(name);
    ranged_[slot] = true;
    return 0;
  }

  int query(int slot) override {
    const hipError_t e = hipEventQuery(event_[slot]);
    if (e == hipErrorNotReady) return 0;
    if (ranged_[slot]) {
      roctxRangeStop(range_[slot]);
      ranged_[slot] = false;
    }
    return e == hipSuccess ? 1 : CLOUD_E_HIP;
  }

 private:
  static size_t frame_bytes(int w, int h) { return ((size_t)w * h * 16 + 255) & ~(size_t)255; }
  size_t scratch_frames() const { return split_ ? 2 : 1; }

  // table (with zeroed counters) -> persistent render [-> batched resolve,
  // on the same queue without a resolve queue]
  hipError_t enqueue_render(int slot) {
    const hipStream_t q = stream_[0];
    hipError_t e = hipMemcpyAsync(dev_[slot], host_[slot], sizeof(ServeTable),
                                  hipMemcpyHostToDevice, q);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn_, dim3(render_blocks_), dim3(256), 0, q, vol_, dev_[slot]->counters,
                       static_cast<const ServeTable*>(dev_[slot]));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return split_ ? hipSuccess : enqueue_resolve(slot);
  }

  hipError_t enqueue_resolve(int slot) {
    hipLaunchKernelGGL(serve_taa_kernel, dim3(taa_blocks_), dim3(256), 0, stream_[split_ ? 1 : 0],
                       dev_[slot]);
    return hipGetLastError();
  }

  // Graph g of slot: 0 the render (with the resolve on one queue), 1 the
  // resolve on the resolve queue.
  hipError_t capture(int slot) {
    for (int g = 0; g < (split_ ? 2 : 1); ++g) {
      const hipStream_t q = stream_[g];
      hipError_t e = hipStreamBeginCapture(q, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return e;
      const hipError_t le = g == 0 ? enqueue_render(slot) : enqueue_resolve(slot);
      e = hipStreamEndCapture(q, &graph_[slot][g]);
      if (le != hipSuccess) return le;
      if (e != hipSuccess) return e;
      if ((e = hipGraphInstantiate(&exec_[slot][g], graph_[slot][g], nullptr, nullptr, 0)) != hipSuccess)
        return e;
    }
    return hipSuccess;
  }

  static int err(hipError_t e, std::string* msg) {
    *msg = std::string("HIP: ") + hipGetErrorString(e);
    return CLOUD_E_HIP;
  }

  int device_;
  DevVolume vol_;
  size_t volume_bytes_;
  float blend_;
  bool graphs_;
  bool split_;
  bool history_in_output_;
  RenderFn fn_ = nullptr;
  int render_blocks_ = 0, taa_blocks_ = 0;
  hipStream_t stream_[2] = {};        // render (and resolve) queue; resolve queue
  hipEvent_t event_[kSlots] = {};     // batch done
  hipEvent_t rendered_[kSlots] = {};  // batch rendered (resolve queue only)
  ServeTable* host_[kSlots] = {};
  ServeTable* dev_[kSlots] = {};
  hipGraph_t graph_[kSlots][2] = {};
  hipGraphExec_t exec_[kSlots][2] = {};
  roctx_range_id_t range_[kSlots] = {};
  bool ranged_[kSlots] = {};
};

}  // namespace
}  // namespace cloud

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

struct cloud_server {
  cloud_volume volume;
  std::unique_ptr<cloud::HipExecutor> ex;
  std::unique_ptr<cloud::serve::Scheduler> sched;
};

using namespace cloud;

extern "C" {

int cloud_serve_create(const cloud_volume* shared, const cloud_serve_config* cfg,
                       cloud_server** out) {
  try {
    clear_error();
    if (!out) return fail(CLOUD_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!cfg) return fail(CLOUD_E_INVALID, "config is NULL");
    if (cfg->max_batch < 1 || cfg->max_batch > kMaxBatch)
      return fail(CLOUD_E_INVALID, "max_batch must be in [1, 64]");
    if (cfg->max_queue < 1) return fail(CLOUD_E_INVALID, "max_queue must be >= 1");
    if (cfg->queues < 0 || cfg->queues > 2) return fail(CLOUD_E_INVALID, "queues must be 0, 1 or 2");
    if (cfg->history_in_output != 0 && cfg->history_in_output != 1)
      return fail(CLOUD_E_INVALID, "history_in_output must be 0 or 1");
    if (cfg->start_lead_us < -1 || cfg->start_lead_us > 1000000)
      return fail(CLOUD_E_INVALID, "start_lead_us must be in [-1, 1000000]");
    if (!std::isfinite(cfg->taa_blend) || !(cfg->taa_blend > 0.0f) || cfg->taa_blend > 1.0f)
      return fail(CLOUD_E_INVALID, "taa_blend must be in (0, 1]");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev)
      return fail(CLOUD_E_INVALID, "no such device");
    if (hipSetDevice(cfg->device) != hipSuccess) return fail(CLOUD_E_HIP, "hipSetDevice failed");
    DevVolume v;
    int dtype, rc;
    if ((rc = prepare_volume(shared, &v, &dtype))) return rc;
    size_t volume_bytes = 0;
    if ((rc = volume_layout_bytes(shared, shared->layout, &volume_bytes))) return rc;
    auto srv = std::make_unique<cloud_server>();
    srv->volume = *shared;
    const int queues = cfg->queues == 0 ? 1 : cfg->queues;
    srv->ex = std::make_unique<HipExecutor>(cfg->device, v, volume_bytes, dtype, shared->layout,
                                            cfg->taa_blend, cfg->use_graphs != 0, queues,
                                            cfg->history_in_output != 0);
    std::string msg;
    if ((rc = srv->ex->init(&msg))) return fail(rc, msg);
    serve::Config sc;
    sc.budget_bytes = cfg->hbm_budget_bytes;
    sc.max_batch = cfg->max_batch;
    sc.max_queue = cfg->max_queue;
    sc.depth = kSlots;
    // renders run in launch order, and so do resolves, each after its
    // batch's render: a stream's next request may follow its previous one in
    // the next batch
    sc.pipeline = kSlots;
    sc.lead_ns = cfg->start_lead_us < 0 ? -1
                 : 1000LL * (cfg->start_lead_us == 0 ? kDefaultStartLeadUs : cfg->start_lead_us);
    srv->sched = std::make_unique<serve::Scheduler>(srv->ex.get(), sc);
    *out = srv.release();
    return CLOUD_OK;
  } catch (const std::bad_alloc&) {
    return fail(CLOUD_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(CLOUD_E_INVALID, "internal error");
  }
}

int cloud_serve_submit(cloud_server* srv, uint64_t stream_id, const cloud_camera* camera,
                       const cloud_params* params, int32_t width, int32_t height,
                       uint32_t frame_index, float* out_rgba, uint64_t* request_id) {
  try {
    clear_error();
    if (!srv) return fail(CLOUD_E_INVALID, "server is NULL");
    if (!request_id) return fail(CLOUD_E_INVALID, "request_id is NULL");
    int rc = check_image(width, height, 1);
    if (rc) return rc;
    Payload pl;
    if ((rc = prepare_camera(camera, width, height, &pl.cam))) return rc;
    if ((rc = prepare_params(params, &srv->volume, &pl.prm))) return rc;
    if (reinterpret_cast<uintptr_t>(out_rgba) % 16)
      return fail(CLOUD_E_INVALID, "out_rgba must be 16-byte aligned");
    if ((rc = check_span(out_rgba, (size_t)width * height * 16, "out_rgba"))) return rc;
    std::vector<unsigned char> bytes(sizeof pl);
    std::memcpy(bytes.data(), &pl, sizeof pl);
    std::string msg;
    rc = srv->sched->submit(stream_id, width, height, frame_index, out_rgba, std::move(bytes),
                            request_id, &msg);
    if (rc) return fail(rc, msg);
    return CLOUD_OK;
  } catch (const std::bad_alloc&) {
    return fail(CLOUD_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(CLOUD_E_INVALID, "internal error");
  }
}

int cloud_serve_poll(cloud_server* srv, cloud_completion* out, int32_t max, int32_t* n_out) {
  try {
    clear_error();
    if (!srv || !n_out || (max > 0 && !out)) return fail(CLOUD_E_INVALID, "NULL argument");
    *n_out = 0;
    // completions move out in chunks through a fixed buffer, so max bounds
    // nothing the library allocates
    constexpr int kChunk = 64;
    serve::Completion tmp[kChunk];
    int total = 0;
    while (total < max) {
      int n = 0;
      srv->sched->poll(tmp, std::min(kChunk, max - total), &n);
      for (int i = 0; i < n; ++i) {
        cloud_completion& c = out[total + i];
        c.request_id = tmp[i].request_id;
        c.stream_id = tmp[i].stream_id;
        c.status = tmp[i].status;
        c.reserved = 0;
        c.t_submit_ns = tmp[i].t_submit;
        c.t_admit_ns = tmp[i].t_admit;
        c.t_start_ns = tmp[i].t_start;
        c.t_done_ns = tmp[i].t_done;
      }
      total += n;
      *n_out = total;
      if (n < kChunk) break;
    }
    return CLOUD_OK;
  } catch (const std::bad_alloc&) {
    return fail(CLOUD_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(CLOUD_E_INVALID, "internal error");
  }
}

int cloud_serve_wait(cloud_server* srv, int64_t timeout_ns) {
  try {
    clear_error();
    if (!srv) return fail(CLOUD_E_INVALID, "server is NULL");
    return srv->sched->wait(timeout_ns);
  } catch (const std::bad_alloc&) {
    return fail(CLOUD_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(CLOUD_E_INVALID, "internal error");
  }
}

int cloud_serve_stats(cloud_server* srv, cloud_serve_stats_t* out) {
  try {
    clear_error();
    if (!srv || !out) return fail(CLOUD_E_INVALID, "NULL argument");
    const serve::Stats s = srv->sched->stats();
    out->queued = s.queued;
    out->admitted = s.admitted;
    out->running = s.running;
    out->completed = s.completed;
    out->rejected = s.rejected;
    out->cancelled = s.cancelled;
    out->failed = s.failed;
    out->streams = s.streams;
    out->bytes_in_use = s.bytes_in_use;
    out->batches = s.batches;
    return CLOUD_OK;
  } catch (const std::bad_alloc&) {
    return fail(CLOUD_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(CLOUD_E_INVALID, "internal error");
  }
}

int cloud_serve_close_stream(cloud_server* srv, uint64_t stream_id) {
  try {
    clear_error();
    if (!srv) return fail(CLOUD_E_INVALID, "server is NULL");
    const int rc = srv->sched->close_stream(stream_id);
    if (rc) return fail(rc, "unknown stream");
    return CLOUD_OK;
  } catch (const std::bad_alloc&) {
    return fail(CLOUD_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(CLOUD_E_INVALID, "internal error");
  }
}

int cloud_serve_destroy(cloud_server* srv) {
  try {
    clear_error();
    if (!srv) return fail(CLOUD_E_INVALID, "server is NULL");
    srv->sched.reset();   // cancels queued requests, waits for in-flight batches
    srv->ex.reset();
    delete srv;
    return CLOUD_OK;
  } catch (const std::bad_alloc&) {
    return fail(CLOUD_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(CLOUD_E_INVALID, "internal error");
  }
}

}  // extern "C"

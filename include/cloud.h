/*
 * cloud.h -- C ABI of the MI355X (gfx950) cloud raymarch library.
 *
 * The library renders the volumetric-cloud method of Toft, Bowles and
 * Zimmermann, "Optimisations for Real-Time Volumetric Cloudscapes"
 * (arXiv 1609.05344): a per-pixel primary raymarch through a 3-D density
 * field (Section 1) with a per-pixel jittered start (Section 3.2), a
 * Beer-Lambert light march towards the sun at each sample, Henyey-Greenstein
 * phase plus an ambient term (Section 1), the analytic integration of
 * scattering over each step (Section 3.1), and a temporal resolve that
 * accumulates the jittered frames (Section 3.2).
 *
 * Conventions shared by every entry point:
 *  - Return value: CLOUD_OK (0) or a negative CLOUD_E_* code. No C++
 *    exception crosses this boundary. cloud_last_error() returns a
 *    thread-local message describing the last non-OK result on the calling
 *    thread.
 *  - Pointers marked "device" are HIP device memory owned by the caller; the
 *    library never frees them and never keeps them beyond the call, except a
 *    server's shared volume (see cloud_serve_create). Struct arguments are
 *    host memory, read during the call only.
 *  - Every argument is checked on the host before anything is launched; an
 *    invalid call returns CLOUD_E_INVALID and launches nothing.
 *  - Render and resolve calls are asynchronous: work is enqueued on the given
 *    HIP stream (a hipStream_t passed as void*, NULL for the default stream)
 *    and the call returns. A launch failure is CLOUD_E_HIP; a fault during
 *    execution surfaces at the caller's next synchronisation.
 *  - Identical inputs give bitwise-identical outputs (no floating-point
 *    atomics; every output element is written by exactly one thread).
 *  - Images are [height][width][4] float32 RGBA, row 0 at the top, 16-byte
 *    aligned. Colour is premultiplied by opacity; alpha = 1 - T, where T is
 *    the transmittance along the view ray. No background is composited.
 */
#ifndef CLOUD_H
#define CLOUD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Raised whenever a struct layout or a signature changes (2: brick_log2 in
 * cloud_volume, queues in cloud_serve_config, depth/trace/composite entry
 * points; 3: the gather record and replay entry points; 4: history_in_output
 * and start_lead_us in cloud_serve_config; 5: cloud_render_resolve). */
#define CLOUD_ABI_VERSION 5

enum {
  CLOUD_OK = 0,
  CLOUD_E_INVALID = -1,   /* bad argument; nothing launched */
  CLOUD_E_NOMEM = -2,     /* allocation failed, or request can never fit a budget */
  CLOUD_E_HIP = -3,       /* HIP runtime error (launch, copy, event) */
  CLOUD_E_BUSY = -4,      /* server queue full; retry later */
  CLOUD_E_NOTFOUND = -5,  /* unknown stream or request id */
  CLOUD_E_CANCELLED = -6  /* request dropped by cloud_serve_destroy */
};

/* Memory layout of a base density volume. Every layout holds the same
 * texel values and gives bitwise-identical renders; the packed layouts
 * replicate each trilinear footprint so that a lookup is one or two aligned
 * fetches instead of eight scattered ones (see cloud_volume_pack).
 *  DENSE  [nz][ny][nx] texels.
 *  QUAD   nz x (ny+1) x (nx+1) entries of 4 texels: entry (z, y', x') holds
 *         the texels (x, y), (x+1, y), (x, y+1), (x+1, y+1) of plane z with
 *         x = x'-1, y = y'-1, indices clamped to the volume (4x storage).
 *  OCT    (nz+1) x (ny+1) x (nx+1) entries of 8 texels: the QUAD entry of
 *         plane z'-1 then that of plane z' (planes clamped; 8x storage).
 * Packed entries are stored in bricks of 8 entries (one 128-byte line of
 * 16-byte entries): 2^bx x 2^by x 2^bz entries with (bx, by, bz) from
 * cloud_volume.brick_log2 (default 1, 1, 1), x fastest inside a brick, then
 * y, then z, bricks in [z][y][x] order, each axis rounded up to whole bricks;
 * cloud_volume_packed_bytes gives the size. The brick shape changes only
 * addresses (renders are bitwise the same); the best shape depends on the
 * workload. */
enum { CLOUD_LAYOUT_DENSE = 0, CLOUD_LAYOUT_QUAD = 1, CLOUD_LAYOUT_OCT = 2 };

/* Storage type of a density volume. Every type is decoded exactly to
 * float32; all optical depth, transmittance, exponentials and colour are
 * accumulated in float32. */
enum { CLOUD_F32 = 0, CLOUD_F16 = 1, CLOUD_BF16 = 2 };

/* Density field (Section 1: "the density is sampled" at each step).
 *  base    device, [nz][ny][nx] values of type dtype, x fastest, y up. Texel
 *          (i,j,k) is centred at box_min + (i+0.5, j+0.5, k+0.5) * extent/n.
 *          Lookups are trilinear (x, then y, then z) with clamp-to-edge.
 *  detail  device, optional (NULL = none), [dnz][dny][dnx] of type ddtype,
 *          tiled detail_tiling times across the box with repeat addressing.
 *          With detail the density is
 *          clamp((b - detail_weight*d) / (1 - detail_weight*d), 0, 1).
 *  layout  CLOUD_LAYOUT_* of base (a packed base is 16-byte aligned and
 *          normally made by cloud_volume_pack); nx, ny, nz always count
 *          texels. In a packed volume the detail, if any, is packed too:
 *          [dnz][dny][dnx] entries of 8 texels, entry (z, y, x) holding the
 *          texels at x|x+1, y|y+1, z|z+1 (each wrapped) in the OCT order,
 *          16-byte aligned (cloud_volume_pack writes it after the base).
 *  occupancy       device, optional (NULL = none): a bitmap made by
 *          cloud_volume_occupancy, one bit per brick of 2^occupancy_log2
 *          texels per axis, clear when every texel a trilinear footprint
 *          starting in that brick can touch is zero. A lookup in a clear
 *          brick is exactly zero, so it is answered without reading the
 *          volume; results are bitwise identical with and without it.
 *  brick_log2      packed layouts: log2 of the brick extent along x, y, z,
 *          each in [0, 3] and summing to 3, or all 0 for (1, 1, 1). A packed
 *          volume must be described with the shape it was packed with
 *          (cloud_volume_pack copies it into the packed descriptor).
 *  Requirements: n* >= 2, dn* >= 2 when detail is set, fewer than 2^24
 *  entries per plane, box_max > box_min on every axis,
 *  0 <= detail_weight < 1, detail_tiling > 0, detail values in [0, 1].
 *  The volume must stay valid until the call's work has run. */
typedef struct {
  const void* base;
  int32_t nx, ny, nz;
  int32_t dtype;
  const void* detail;
  int32_t dnx, dny, dnz;
  int32_t ddtype;
  float detail_weight;
  float detail_tiling;
  float box_min[3];
  float box_max[3];
  int32_t layout;
  const uint32_t* occupancy;
  int32_t occupancy_log2;
  int32_t brick_log2[3];  /* packed layouts: brick shape (see above); all 0 = 1, 1, 1 */
} cloud_volume;

/* Pinhole camera: rays leave pos through pixel centres; vfov_deg is the
 * vertical field of view; up fixes the roll (it must not be parallel to
 * target - pos). */
typedef struct {
  float pos[3];
  float target[3];
  float up[3];
  float vfov_deg;
} cloud_camera;

/* Method parameters.
 *  steps        N primary samples over the ray's chord through the box, at
 *               t_near + (i + j) * D, D = chord / N (Sections 1 and 3.2).
 *  light_steps  L samples of the march towards the sun (Section 1), at the
 *               midpoints of L equal steps to the box exit; 0 disables it.
 *  alpha        extinction per unit density (the paper's "absorption"), >= 0.
 *  g            Henyey-Greenstein asymmetry, |g| < 1 (Section 1).
 *  sun_dir      direction towards the sun (any non-zero length).
 *  sun_color    light colour times intensity, per channel.
 *  ambient      ambient light added to the incident light (Section 1).
 *  jitter       0: j = 0.5 for every ray; 1: per-pixel offset j in [0, 1)
 *               from the PCG hash chain of (px, py, frame_index, seed)
 *               (Section 3.2's random per-pixel start offset); 2: one offset
 *               per 8x8-pixel tile, the chain of (px >> 3, py >> 3, ...);
 *               3: one offset per frame, the chain of (0, 0, ...). Modes 2
 *               and 3 are coherent variants (the cache-friendlier jitter
 *               Section 5 leaves to future work).
 *  integration  1: analytic, S += T L_in (1 - exp(-rho alpha D)) (Section 3.1);
 *               0: the basic rule, T updated first, S += T rho alpha D L_in.
 *  t_eps        stop a ray once T < t_eps (the march ends once the alpha is
 *               full, Section 1); 0 disables the early exit. */
typedef struct {
  int32_t steps;
  int32_t light_steps;
  float alpha;
  float g;
  float sun_dir[3];
  float sun_color[3];
  float ambient[3];
  int32_t jitter;
  uint32_t seed;
  int32_t integration;
  float t_eps;
} cloud_params;

/* Thread-local description of the last error on this thread ("" if none). */
const char* cloud_last_error(void);

/* CLOUD_ABI_VERSION of the loaded library. */
int cloud_abi_version(void);

/* Render one frame of the cloud layer (Sections 1, 3.1, 3.2).
 *  out_rgba   device [height][width][4] float32, written completely (rays
 *             that miss the box get 0).
 *  frame_index feeds the jitter hash. width, height >= 1. */
int cloud_render(const cloud_volume* volume, const cloud_camera* camera,
                 const cloud_params* params, uint32_t frame_index,
                 int32_t width, int32_t height, float* out_rgba,
                 void* hip_stream);

/* Render n_views cameras of one volume in one launch (same size, params and
 * frame_index). cameras is a host array of n_views; out_rgba is device
 * [n_views][height][width][4]. View v's pixels hash exactly as in
 * cloud_render. n_views >= 1. */
int cloud_render_views(const cloud_volume* volume, const cloud_camera* cameras,
                       int32_t n_views, const cloud_params* params,
                       uint32_t frame_index, int32_t width, int32_t height,
                       float* out_rgba, void* hip_stream);

/* March n explicit rays (same method as cloud_render; used to check single
 * rays against closed forms).
 *  origins, dirs  device [n][3] float32; dirs are normalised by the library
 *                 and must be non-zero.
 *  pixel_xy       device [n][2] uint32 (px, py) fed to the jitter hash
 *                 (under params->jitter's mode), or NULL for j = 0.5;
 *                 ignored when params->jitter == 0.
 *  out_rgba       device [n][4] float32. n == 0 is a no-op. */
int cloud_march_rays(const cloud_volume* volume, const float* origins,
                     const float* dirs, const uint32_t* pixel_xy, int64_t n,
                     const cloud_params* params, uint32_t frame_index,
                     float* out_rgba, void* hip_stream);

/* Temporal resolve of a jittered frame (Section 3.2): for each pixel and
 * channel, clamp the history into the min/max of the current frame's 3x3
 * neighbourhood (edges clamped), then out = h + blend * (current - h).
 * history == NULL or frame_index == 0 copies current to out.
 *  current, history, out  device [height][width][4] float32.
 *  out may equal history (in-place update); out must not overlap current.
 *  0 < blend <= 1. */
int cloud_taa_resolve(const float* current, const float* history, float* out,
                      int32_t width, int32_t height, float blend,
                      uint32_t frame_index, void* hip_stream);

/* cloud_render plus each pixel's representative depth (for the reprojected
 * resolve): out_depth (device [height][width] float32, 4-byte aligned,
 * caller-owned, not overlapping out_rgba) gets the mean distance along the
 * ray of the samples, weighted by the opacity each step adds (T before the
 * step minus T after it), where the pixel's alpha >= 0.01; the middle of the
 * ray's chord through the box where alpha < 0.01; 0 (a point at infinity)
 * where the ray misses the box. The image equals cloud_render's. */
int cloud_render_depth(const cloud_volume* volume, const cloud_camera* camera,
                       const cloud_params* params, uint32_t frame_index,
                       int32_t width, int32_t height, float* out_rgba,
                       float* out_depth, void* hip_stream);

/* The render of one frame and the temporal resolve of the frame before it
 * in one launch (Sections 1, 3.1, 3.2), for callers that render frame f
 * while frame f - 1 is still to be resolved: exactly
 * cloud_render_views(volume, cameras, n_views, params, frame_index, width,
 * height, out_rgba) and, for each view v, cloud_taa_resolve(prev_rgba[v],
 * history[v], resolved[v], width, height, blend, prev_frame_index), with
 * bitwise the same results, but the resolve's workgroups are scheduled after
 * the render's, so they run while the render's last tiles finish (up to 16
 * views a launch; more are split into launches of 16). The two parts run
 * concurrently: out_rgba must not overlap prev_rgba, history or resolved, and
 * resolved must not overlap prev_rgba (it may equal history). out_rgba,
 * prev_rgba (the previous frame's render), history and resolved are device
 * [n_views][height][width][4] float32; history == NULL or prev_frame_index
 * == 0 copies prev_rgba to resolved. n_views >= 1. */
int cloud_render_resolve(const cloud_volume* volume, const cloud_camera* cameras,
                         int32_t n_views, const cloud_params* params,
                         uint32_t frame_index, int32_t width, int32_t height,
                         float* out_rgba, const float* prev_rgba,
                         const float* history, float* resolved, float blend,
                         uint32_t prev_frame_index, void* hip_stream);

/* Temporal resolve with camera reprojection (Section 3.2 names Playdead's
 * TAA, whose history is reprojected). For each pixel, the point at its depth
 * (from cloud_render_depth with `camera`) along its ray -- the ray's
 * direction alone where depth is 0 -- is projected into prev_camera, the
 * camera `history` was resolved with; the history is sampled there
 * bilinearly with edge clamping, clamped into the current frame's 3x3
 * neighbourhood min/max and blended, out = h + blend * (current - h). Where
 * the point is behind prev_camera or outside its image the history is taken
 * to be the current value. frame_index == 0 or history == NULL copies
 * current (depth and cameras are then not read).
 *  current, history, out  device [height][width][4] float32, 16-byte aligned.
 *  depth                  device [height][width] float32.
 *  out must not overlap current, history or depth (no in-place update: a
 *  pixel reads the history at other pixels). 0 < blend <= 1. */
int cloud_taa_resolve_reproject(const float* current, const float* depth,
                                const float* history, float* out,
                                const cloud_camera* camera,
                                const cloud_camera* prev_camera,
                                int32_t width, int32_t height, float blend,
                                uint32_t frame_index, void* hip_stream);

/* Composites a resolved cloud layer into the scene (Section 3.2: the
 * clouds are rendered and resolved in a low-resolution buffer, then
 * composited into the rest of the frame). The layer (premultiplied RGBA,
 * cloud_width x cloud_height) is up-sampled bilinearly to width x height with
 * pixel centres aligned -- output pixel x samples the layer at
 * (x + 1/2) * cloud_width / width - 1/2, likewise in y, edge-clamped -- then
 * out = c + (1 - c.alpha) * background in every channel.
 *  cloud                device [cloud_height][cloud_width][4] float32.
 *  background, out      device [height][width][4] float32.
 * All 16-byte aligned. out may be background itself (in place) but must not
 * overlap it otherwise, nor overlap cloud. */
int cloud_composite(const float* cloud, int32_t cloud_width, int32_t cloud_height,
                    const float* background, float* out, int32_t width,
                    int32_t height, void* hip_stream);

/* Adds to *out_count (device, one uint64, 8-byte aligned) the number of
 * trilinear density lookups cloud_render performs for this frame: one per
 * primary sample taken plus light_steps per sample with non-zero density,
 * up to each ray's early exit. Writes no image. Used to report executed
 * samples per second. */
int cloud_count_lookups(const cloud_volume* volume, const cloud_camera* camera,
                        const cloud_params* params, uint32_t frame_index,
                        int32_t width, int32_t height, uint64_t* out_count,
                        void* hip_stream);

/* Records which lookups cloud_render_views performs for these views and
 * this frame: out_trace (device [n_views][height][width][2] uint32, 8-byte
 * aligned, caller-owned) gets per pixel the number of primary samples taken
 * (up to the early exit, Section 1) and a mask whose bit i is set when
 * sample i ran the light march (density > 0). Requires params->steps <= 32.
 * Writes no image. Input to cloud_gather_record. */
int cloud_lookup_trace(const cloud_volume* volume, const cloud_camera* cameras,
                       int32_t n_views, const cloud_params* params,
                       uint32_t frame_index, int32_t width, int32_t height,
                       uint32_t* out_trace, void* hip_stream);

/* Measurement only (Sections 4 and 5: the per-pixel jitter costs the render
 * cache misses, so its achievable speed is set by its own gather pattern).
 * Records every density lookup a cloud_render_views of these views makes, as
 * the texel corner of the lookup's footprint, in the order each wavefront
 * issues them. A wavefront's lookup instructions are its slots: step i's
 * primary lookup while any of its lanes still marches, then the light
 * march's lookups if any lane ran it at step i.
 *  codes: device uint32 [n_waves][max_slots][64], n_waves = n_views *
 *         ceil(width/16) * ceil(height/16) * 4 (wavefronts in the render's
 *         block order, view-major); per lane of a slot kx | ky << 10 |
 *         kz << 20, with bit 30 set when the occupancy skip redirects the
 *         fetch to entry 0, or 0xFFFFFFFF when the lane makes no lookup in
 *         the slot. Slots past a wavefront's count are not written.
 *  slot_counts: device uint32 [n_waves], the slots each wavefront used.
 *  max_slots >= steps * (1 + light_steps); trace from cloud_lookup_trace for
 *  the same volume, cameras, params and frame (8-byte aligned).
 * Volumes of at most 1024 texels per axis, no detail volume, steps <= 32. */
int cloud_gather_record(const cloud_volume* volume, const cloud_camera* cameras,
                        int32_t n_views, const cloud_params* params,
                        uint32_t frame_index, int32_t width, int32_t height,
                        const uint32_t* trace, int32_t max_slots, uint32_t* codes,
                        uint32_t* slot_counts, void* hip_stream);

/* Measurement only: the fetch-only replay of a recorded pattern. One launch on
 * the render's launch shape and tile walk; each wavefront takes its slots in
 * order and fetches the volume words of each lane's corner (the entry index
 * of the volume's layout; entry 0 for a redirected corner), with no camera,
 * jitter, ray-box, light-path, interpolation or lighting arithmetic:
 *  mode 0: the recorded corners;
 *  mode 1: a uniformly random corner of the whole volume for each recorded
 *          lookup (same slots and lanes, no redirect).
 * blocks_per_cu caps resident workgroups per CU (0: no cap; a cap the device
 * cannot reach with LDS is CLOUD_E_INVALID). out: device uint32
 * [n_waves][64], an XOR of the words each lane fetched (no meaning; it keeps
 * every fetch). volume: the one the codes were recorded on, in any layout.
 * Corners are clamped into the volume and slot counts to max_slots whatever
 * the buffers hold. */
int cloud_gather_replay(const cloud_volume* volume, int32_t n_views, int32_t width,
                        int32_t height, const uint32_t* codes, int32_t max_slots,
                        const uint32_t* slot_counts, int32_t mode, int32_t blocks_per_cu,
                        uint32_t* out, void* hip_stream);

/* Device bytes a copy of the dense volume's base needs in `layout`. */
int cloud_volume_packed_bytes(const cloud_volume* dense, int32_t layout,
                              uint64_t* bytes);

/* Enqueues the repacking of dense->base (layout CLOUD_LAYOUT_DENSE) into dst
 * in layout CLOUD_LAYOUT_QUAD or CLOUD_LAYOUT_OCT, and fills *packed with
 * dense's descriptor re-pointed at dst. dst: device, caller-owned,
 * 16-byte aligned, at least cloud_volume_packed_bytes bytes (dst_bytes), not
 * overlapping the source. Values are copied bit for bit, so renders of the
 * packed and dense volumes are identical. */
int cloud_volume_pack(const cloud_volume* dense, int32_t layout, void* dst,
                      uint64_t dst_bytes, cloud_volume* packed, void* hip_stream);

/* Occupancy bitmap of the dense volume's base, for exact empty-space
 * skipping (see cloud_volume.occupancy). The brick size is the smallest
 * power of two >= 4 texels for which the bitmap has at most 32768 bits, so
 * that the kernels can keep it in LDS. *bytes / *log2_brick receive the
 * bitmap size and brick size. */
int cloud_volume_occupancy_bytes(const cloud_volume* dense, uint64_t* bytes,
                                 int32_t* log2_brick);

/* Enqueues the build of that bitmap into dst (device, caller-owned, at
 * least cloud_volume_occupancy_bytes bytes, 4-byte aligned) and fills
 * *with_occupancy with the volume's descriptor pointing at it (any layout of
 * the same texels may then use it). Bit b of word w is brick w*32+b, bricks
 * ordered x fastest. */
int cloud_volume_occupancy(const cloud_volume* dense, uint32_t* dst, uint64_t dst_bytes,
                           cloud_volume* with_occupancy, void* hip_stream);

/* Launch-shape knob, process-wide, for tuning and benchmarking; results do
 * not depend on it. Keys:
 *  "supertile" (-1..64, default -1 = 4) -- the render walks its 16x16-pixel
 *      tiles in S x S super-tiles (0 = row-major).
 *  "xcd_run" (-1..65536, default -1 = S * S) -- the walk is dealt to the 8
 *      XCDs in rounds of runs of this many tiles (XCD x takes run
 *      (x + 3j) mod 8 of round j), so that every XCD's share is spread over
 *      the image (equal work) yet made of compact runs (shared L2); 0 gives
 *      each XCD one contiguous eighth of the walk.
 *  "taa_tile" (16, 32 or 64, default 32) -- the resolve's tile width in
 *      pixels (each tile holds 256 pixels).
 *  "render_blocks_per_cu" (0..64, default 0 = no cap) -- at most this many
 *      render workgroups resident per CU, enforced by reserving LDS at
 *      launch (CLOUD_E_INVALID when the device's LDS cannot express it).
 *  "serve_blocks_per_cu" (0..64, default 0 = automatic: 4 for a stored
 *      volume above 512 MiB, else as many as fit) -- the persistent serving
 *      render's workgroups per CU, read by cloud_serve_create. */
int cloud_tune(const char* key, int32_t value);

/* Checks that [ptr, ptr + bytes) lies inside one HIP device allocation: the
 * check every entry point applies to its buffers before launching anything.
 * Returns CLOUD_OK or CLOUD_E_INVALID (NULL, host memory, or a range that
 * runs past the end of its allocation). Launches nothing. */
int cloud_check_buffer(const void* ptr, uint64_t bytes);

/* The per-pixel start offsets the renderer draws (Section 3.2's random
 * offset), exposed so callers can reproduce a frame's sample positions:
 * out_bits[i] = j * 2^24 (an integer below 2^24) for pixel
 * (pixel_xy[2i], pixel_xy[2i+1]) at frame_index and seed.
 *  pixel_xy device [n][2] uint32; out_bits device [n] uint32; n == 0 is a
 *  no-op. */
int cloud_jitter_offsets(const uint32_t* pixel_xy, int64_t n, uint32_t frame_index,
                         uint32_t seed, uint32_t* out_bits, void* hip_stream);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of render requests from many camera streams
 * (each request is one jittered frame of Section 3.2 plus its temporal
 * resolve against the stream's history).
 *
 * A server shares one volume between all streams. cloud_serve_submit queues
 * a request and returns at once; a scheduler thread admits queued requests
 * into batches as batch slots and device memory allow, and runs each batch as
 * one persistent render launch plus one batched resolve launch (replayed from
 * a captured HIP graph). Up to two batches are in flight, so requests that
 * arrive while the device works are admitted into the next batch; with a
 * batch in flight, the next one starts shortly before the work ahead of it is
 * expected to end (start_lead_us), and admits arrivals until then. A stream's
 * frames run in submission order, one per batch (they chain through the
 * history), and a stream may have two requests in flight, in consecutive
 * batches. Requests of different streams overlap.
 * Results are bitwise identical to cloud_render followed by cloud_taa_resolve
 * on the same inputs, whatever else is in the batch. A request that resolves
 * against the history of a failed request fails too.
 *
 * Stream state is library-owned: a scratch frame (two with queues = 2),
 * plus, unless history_in_output is set, the history (width x height x 16
 * bytes each, rounded up to 256 bytes). It is allocated when the stream's
 * first request is admitted, counted against hbm_budget_bytes, and freed by
 * cloud_serve_close_stream or cloud_serve_destroy. A stream's resolution is fixed by its first request.
 * frame_index 0 (or a stream without valid history) copies the rendered frame
 * instead of resolving it.
 *
 * Thread safety: submit, poll, wait and stats may be called from any thread
 * concurrently; create, close_stream and destroy must not race with other
 * calls on the same server. Timestamps are CLOCK_MONOTONIC nanoseconds.
 * ------------------------------------------------------------------------ */

typedef struct cloud_server cloud_server;

typedef struct {
  uint64_t hbm_budget_bytes;  /* device memory for stream state */
  int32_t max_batch;          /* requests per batch, 1..64 */
  int32_t max_queue;          /* queued (not yet admitted) requests, >= 1 */
  int32_t device;             /* HIP device ordinal */
  float taa_blend;            /* resolve blend, (0, 1] */
  int32_t use_graphs;         /* 1: replay captured graphs; 0: plain launches */
  int32_t queues;             /* 1 (0 means 1): a batch's table copy, render
                               * and resolve run in order on one HIP stream; 2:
                               * resolves run on a second stream, each after
                               * its batch's render and the previous resolve,
                               * overlapping the next batch's render (stream
                               * state then holds two scratch frames) */
  int32_t history_in_output;  /* 1: a stream's history is its previous frame's
                               * output buffer, not a library copy: each
                               * resolved pixel is written once, and the caller
                               * leaves a frame's output unmodified until the
                               * stream's next frame has completed (one buffer
                               * for every frame of a stream is allowed; it is
                               * then resolved in place). 0: the library keeps
                               * the history. */
  int32_t start_lead_us;      /* with a batch in flight, the next starts when
                               * the work ahead is expected to end within this
                               * many microseconds plus an eighth of that work;
                               * 0: the default (300); -1: as soon as a slot is
                               * free */
} cloud_serve_config;

typedef struct {
  uint64_t queued, admitted, running, completed, rejected, cancelled, failed;
  uint64_t streams, bytes_in_use, batches;
} cloud_serve_stats_t;

typedef struct {
  uint64_t request_id, stream_id;
  int32_t status;     /* CLOUD_OK, CLOUD_E_CANCELLED, CLOUD_E_HIP, CLOUD_E_NOMEM */
  int32_t reserved;
  int64_t t_submit_ns, t_admit_ns, t_start_ns, t_done_ns;
} cloud_completion;

/* Creates a server on cfg->device sharing `shared` (device memory that must
 * outlive the server; any layout and dtype). */
int cloud_serve_create(const cloud_volume* shared, const cloud_serve_config* cfg,
                       cloud_server** out);

/* Queues one frame of stream stream_id. out_rgba: device [height][width][4]
 * float32, caller-owned, 16-byte aligned, not touched by the caller until
 * the request completes (with history_in_output: not written by the caller
 * until the stream's next request completes; it may be read once this one
 * has). Returns CLOUD_E_BUSY when the queue is full (retry later),
 * CLOUD_E_NOMEM when this stream's state can never fit the budget,
 * CLOUD_E_INVALID for bad arguments or a resolution that differs from the
 * stream's first request. Camera and params are copied. */
int cloud_serve_submit(cloud_server* server, uint64_t stream_id,
                       const cloud_camera* camera, const cloud_params* params,
                       int32_t width, int32_t height, uint32_t frame_index,
                       float* out_rgba, uint64_t* request_id);

/* Moves up to max finished requests into out (host array of at least max
 * entries); *n_out gets the count. Never blocks, and allocates nothing that
 * grows with max (completions move through a fixed 64-entry buffer), so any
 * max, however large, returns a code. */
int cloud_serve_poll(cloud_server* server, cloud_completion* out, int32_t max,
                     int32_t* n_out);

/* Blocks until at least one completion can be polled or timeout_ns passes.
 * Returns 1 if completions are ready, 0 on timeout, or a CLOUD_E_* code. */
int cloud_serve_wait(cloud_server* server, int64_t timeout_ns);

int cloud_serve_stats(cloud_server* server, cloud_serve_stats_t* out);

/* Cancels the stream's queued requests (they complete as CLOUD_E_CANCELLED)
 * and frees its state once its in-flight requests, if any, have finished.
 * CLOUD_E_NOTFOUND for an unknown stream. */
int cloud_serve_close_stream(cloud_server* server, uint64_t stream_id);

/* Cancels queued requests, waits for in-flight batches, frees everything. */
int cloud_serve_destroy(cloud_server* server);

#ifdef __cplusplus
}
#endif

#endif /* CLOUD_H */

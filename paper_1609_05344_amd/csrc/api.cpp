// C ABI entry points: argument checks, conversion to launch form, launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <string>

#include "../../include/cloud.h"
#include "cloud_launch.h"
#include "cloud_prepare.h"

namespace cloud {

static thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

void clear_error() { g_last_error.clear(); }

size_t dtype_size(int dtype) {
  switch (dtype) {
    case CLOUD_F32: return 4;
    case CLOUD_F16: return 2;
    case CLOUD_BF16: return 2;
    default: return 0;
  }
}

static bool finite3(const float* v) {
  return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

int check_span(const void* p, size_t bytes, const char* what) {
  if (p == nullptr) return fail(CLOUD_E_INVALID, std::string(what) + " is NULL");
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) == hipSuccess && base) {
    const char* b = static_cast<const char*>(base);
    const char* q = static_cast<const char*>(p);
    if (q < b || (size_t)(q - b) + bytes > size) {
      char buf[256];
      snprintf(buf, sizeof buf, "%s: %zu bytes at offset %zu exceed its %zu-byte allocation",
               what, bytes, (size_t)(q - b), size);
      return fail(CLOUD_E_INVALID, buf);
    }
    return CLOUD_OK;
  }
  (void)hipGetLastError();
  return fail(CLOUD_E_INVALID, std::string(what) + " is not inside a device allocation");
}

int check_image(int W, int H, long long views) {
  if (W < 1 || H < 1) return fail(CLOUD_E_INVALID, "width and height must be >= 1");
  if (W > 65536 || H > 65536) return fail(CLOUD_E_INVALID, "width and height must be <= 65536");
  const long long tiles = (long long)((W + 15) / 16) * ((H + 15) / 16) * views;
  if (tiles > 0x7FFFFFFFLL) return fail(CLOUD_E_INVALID, "image too large");
  return CLOUD_OK;
}

// Brick shifts of a volume's packed entries (all zero means 1, 1, 1); false
// when the shape is not one of 8 entries with every shift in [0, 3].
bool brick_shape(const cloud_volume* v, int b[3]) {
  const int* s = v->brick_log2;
  if (s[0] == 0 && s[1] == 0 && s[2] == 0) {
    b[0] = b[1] = b[2] = 1;
    return true;
  }
  for (int k = 0; k < 3; ++k) {
    if (s[k] < 0 || s[k] > 3) return false;
    b[k] = s[k];
  }
  return b[0] + b[1] + b[2] == 3;
}

int volume_layout_bytes(const cloud_volume* v, int layout, size_t* bytes) {
  if (!v) return fail(CLOUD_E_INVALID, "volume is NULL");
  if (layout < CLOUD_LAYOUT_DENSE || layout > CLOUD_LAYOUT_OCT)
    return fail(CLOUD_E_INVALID, "unknown volume layout");
  if (dtype_size(v->dtype) == 0) return fail(CLOUD_E_INVALID, "unknown volume dtype");
  if (v->nx < 2 || v->ny < 2 || v->nz < 2) return fail(CLOUD_E_INVALID, "volume dims must be >= 2");
  // entries (texels, or packed footprints) per plane and in total
  const long long ex = layout == CLOUD_LAYOUT_DENSE ? v->nx : (long long)v->nx + 1;
  const long long ey = layout == CLOUD_LAYOUT_DENSE ? v->ny : (long long)v->ny + 1;
  const long long ez = layout == CLOUD_LAYOUT_OCT ? (long long)v->nz + 1 : v->nz;
  if (ex * ey >= (1LL << 24)) return fail(CLOUD_E_INVALID, "volume planes must hold < 2^24 texels");
  long long row, plane, entries = ex * ey * ez;
  if (layout != CLOUD_LAYOUT_DENSE) {
    int b[3];
    if (!brick_shape(v, b))
      return fail(CLOUD_E_INVALID, "brick_log2 must be three shifts in [0, 3] summing to 3, or all 0");
    packed_strides(ex, ey, ez, b[0], b[1], b[2], &row, &plane, &entries);
  }
  if (entries > 0x7FFFFFFFLL) return fail(CLOUD_E_INVALID, "volume has too many texels");
  const int corners = layout == CLOUD_LAYOUT_DENSE ? 1 : layout == CLOUD_LAYOUT_QUAD ? 4 : 8;
  *bytes = (size_t)entries * corners * dtype_size(v->dtype);
  return CLOUD_OK;
}

// Brick counts of an occupancy bitmap with bricks of 2^lg texels.
static void occupancy_dims(const cloud_volume* v, int lg, int* nbx, int* nby, int* nbz) {
  *nbx = ((v->nx - 1) >> lg) + 1;
  *nby = ((v->ny - 1) >> lg) + 1;
  *nbz = ((v->nz - 1) >> lg) + 1;
}

static int occupancy_words(int nbx, int nby, int nbz) {
  return (int)(((long long)nbx * nby * nbz + 31) / 32);
}

// Smallest brick (>= 4 texels) whose bitmap fits the kernels' LDS budget.
static int occupancy_log2(const cloud_volume* v) {
  for (int lg = 2; lg < 16; ++lg) {
    int a, b, c;
    occupancy_dims(v, lg, &a, &b, &c);
    if (occupancy_words(a, b, c) <= kOccupancyWords) return lg;
  }
  return 16;
}

int prepare_volume(const cloud_volume* v, DevVolume* out, int* dtype) {
  if (!v) return fail(CLOUD_E_INVALID, "volume is NULL");
  size_t bytes = 0;
  int rc = volume_layout_bytes(v, v->layout, &bytes);
  if (rc) return rc;
  for (int k = 0; k < 3; ++k) {
    if (!std::isfinite(v->box_min[k]) || !std::isfinite(v->box_max[k]) ||
        !(v->box_max[k] > v->box_min[k]))
      return fail(CLOUD_E_INVALID, "box_max must exceed box_min on every axis");
  }
  if (v->layout != CLOUD_LAYOUT_DENSE && reinterpret_cast<uintptr_t>(v->base) % 16)
    return fail(CLOUD_E_INVALID, "a packed volume must be 16-byte aligned");
  if ((rc = check_span(v->base, bytes, "volume base"))) return rc;
  DevVolume d = {};
  d.base = v->base;
  d.nx = v->nx; d.ny = v->ny; d.nz = v->nz;
  if (v->layout == CLOUD_LAYOUT_DENSE) {
    d.row = v->nx;
    d.plane = v->nx * v->ny;
  } else {
    int b[3];
    brick_shape(v, b);   // validated by volume_layout_bytes
    long long row, plane, entries;
    packed_strides(v->nx + 1, v->ny + 1, v->layout == CLOUD_LAYOUT_OCT ? v->nz + 1 : v->nz, b[0],
                   b[1], b[2], &row, &plane, &entries);
    d.row = (int)row;
    d.plane = (int)plane;
    d.bx = b[0];
    d.by = b[1];
    d.bz = b[2];
    const int corners = v->layout == CLOUD_LAYOUT_OCT ? 8 : 4;
    d.entry_shift = corners * (int)dtype_size(v->dtype) == 32 ? 5 : corners * (int)dtype_size(v->dtype) == 16 ? 4 : 3;
    d.tab = tab_fits(v->nx, v->ny, v->nz) && bytes <= 0xFFFFFF00ull ? 1 : 0;
    d.tab_bytes = d.tab ? (uint32_t)bytes : 0u;
  }
  const int n[3] = {v->nx, v->ny, v->nz};
  float* s[3] = {&d.sx, &d.sy, &d.sz};
  float* o[3] = {&d.ox, &d.oy, &d.oz};
  for (int k = 0; k < 3; ++k) {
    const double sc = (double)n[k] / ((double)v->box_max[k] - (double)v->box_min[k]);
    *s[k] = (float)sc;
    *o[k] = (float)(-(double)v->box_min[k] * sc - 0.5);
    d.bmin[k] = v->box_min[k];
    d.bmax[k] = v->box_max[k];
  }
  d.detail = nullptr;
  if (v->detail) {
    if (v->ddtype != v->dtype)
      return fail(CLOUD_E_INVALID, "detail dtype must equal the base dtype");
    if (v->dnx < 2 || v->dny < 2 || v->dnz < 2)
      return fail(CLOUD_E_INVALID, "detail dims must be >= 2");
    const long long dt = (long long)v->dnx * v->dny * v->dnz;
    if (dt > 0x7FFFFFFFLL) return fail(CLOUD_E_INVALID, "detail volume too large");
    if (!std::isfinite(v->detail_weight) || v->detail_weight < 0.0f || v->detail_weight >= 1.0f)
      return fail(CLOUD_E_INVALID, "detail_weight must be in [0, 1)");
    if (!std::isfinite(v->detail_tiling) || !(v->detail_tiling > 0.0f))
      return fail(CLOUD_E_INVALID, "detail_tiling must be > 0");
    if ((long long)v->dnx * v->dny >= (1LL << 24))
      return fail(CLOUD_E_INVALID, "detail planes must hold < 2^24 texels");
    // a packed volume keeps its detail in the oct-wrap form (8 texels per texel)
    const bool packed = v->layout != CLOUD_LAYOUT_DENSE;
    if (packed && reinterpret_cast<uintptr_t>(v->detail) % 16)
      return fail(CLOUD_E_INVALID, "a packed detail volume must be 16-byte aligned");
    rc = check_span(v->detail, (size_t)dt * dtype_size(v->ddtype) * (packed ? 8 : 1),
                    "volume detail");
    if (rc) return rc;
    d.detail = v->detail;
    d.dnx = v->dnx; d.dny = v->dny; d.dnz = v->dnz;
    auto pow2 = [](int n) { return (n & (n - 1)) == 0; };
    d.dpow2 = pow2(v->dnx) && pow2(v->dny) && pow2(v->dnz);
    const int dn[3] = {v->dnx, v->dny, v->dnz};
    float* ds[3] = {&d.dsx, &d.dsy, &d.dsz};
    float* dof[3] = {&d.dox, &d.doy, &d.doz};
    for (int k = 0; k < 3; ++k) {
      const double sc = (double)dn[k] * (double)v->detail_tiling /
                        ((double)v->box_max[k] - (double)v->box_min[k]);
      *ds[k] = (float)sc;
      *dof[k] = (float)(-(double)v->box_min[k] * sc - 0.5);
    }
    d.detail_weight = v->detail_weight;
  }
  d.occ = nullptr;
  if (v->occupancy) {
    if (v->occupancy_log2 < 0 || v->occupancy_log2 > 15)
      return fail(CLOUD_E_INVALID, "occupancy_log2 must be in [0, 15]");
    int nbx, nby, nbz;
    occupancy_dims(v, v->occupancy_log2, &nbx, &nby, &nbz);
    const int words = occupancy_words(nbx, nby, nbz);
    if (words > kOccupancyWords)
      return fail(CLOUD_E_INVALID, "occupancy bitmap exceeds 32768 bricks; use a larger brick");
    if (reinterpret_cast<uintptr_t>(v->occupancy) % 4)
      return fail(CLOUD_E_INVALID, "occupancy must be 4-byte aligned");
    if ((rc = check_span(v->occupancy, (size_t)words * 4, "occupancy"))) return rc;
    d.occ = v->occupancy;
    d.occ_lg = v->occupancy_log2;
    d.occ_nbx = nbx;
    d.occ_plane = nbx * nby;
    d.occ_words = words;
  }
  *out = d;
  *dtype = v->dtype;
  return CLOUD_OK;
}

int prepare_params(const cloud_params* p, const cloud_volume* v, DevParams* out) {
  if (!p) return fail(CLOUD_E_INVALID, "params is NULL");
  if (p->steps < 1 || p->steps > (1 << 20)) return fail(CLOUD_E_INVALID, "steps must be in [1, 2^20]");
  if (p->light_steps < 0 || p->light_steps > 4096)
    return fail(CLOUD_E_INVALID, "light_steps must be in [0, 4096]");
  if (!std::isfinite(p->alpha) || p->alpha < 0.0f) return fail(CLOUD_E_INVALID, "alpha must be finite and >= 0");
  if (!std::isfinite(p->g) || !(std::fabs(p->g) < 1.0f)) return fail(CLOUD_E_INVALID, "|g| must be < 1");
  if (!finite3(p->sun_dir) || !finite3(p->sun_color) || !finite3(p->ambient))
    return fail(CLOUD_E_INVALID, "sun_dir, sun_color and ambient must be finite");
  const double sl = std::sqrt((double)p->sun_dir[0] * p->sun_dir[0] +
                              (double)p->sun_dir[1] * p->sun_dir[1] +
                              (double)p->sun_dir[2] * p->sun_dir[2]);
  if (!(sl > 0.0)) return fail(CLOUD_E_INVALID, "sun_dir must be non-zero");
  if (p->jitter < 0 || p->jitter > 3) return fail(CLOUD_E_INVALID, "jitter must be 0, 1, 2 or 3");
  if (p->integration != 0 && p->integration != 1)
    return fail(CLOUD_E_INVALID, "integration must be 0 (naive) or 1 (analytic)");
  if (!std::isfinite(p->t_eps) || p->t_eps < 0.0f) return fail(CLOUD_E_INVALID, "t_eps must be finite and >= 0");
  DevParams d = {};
  d.steps = p->steps;
  d.light_steps = p->light_steps;
  d.alpha = p->alpha;
  d.alpha_log2e = (float)((double)p->alpha * 1.4426950408889634);
  d.inv_light_steps = p->light_steps > 0 ? (float)(1.0 / p->light_steps) : 0.0f;
  for (int k = 0; k < 3; ++k) {
    const double sk = (double)p->sun_dir[k] / sl;
    d.s[k] = (float)sk;
    d.s_axis[k] = d.s[k] != 0.0f;
    d.inv_s[k] = d.s_axis[k] ? (float)(1.0 / (double)d.s[k]) : 0.0f;
    d.light_bound[k] = d.s[k] > 0.0f ? v->box_max[k] : v->box_min[k];
    d.sun[k] = p->sun_color[k];
    d.amb[k] = p->ambient[k];
  }
  const double g = p->g;
  d.hg_k = (float)((1.0 - g * g) / (4.0 * M_PI));
  d.hg_a = (float)(1.0 + g * g);
  d.hg_b = (float)(2.0 * g);
  d.jitter = p->jitter;
  d.seed = p->seed;
  d.integration = p->integration;
  d.t_eps = p->t_eps;
  *out = d;
  return CLOUD_OK;
}

int prepare_camera(const cloud_camera* c, int W, int H, DevCamera* out) {
  if (!c) return fail(CLOUD_E_INVALID, "camera is NULL");
  if (!finite3(c->pos) || !finite3(c->target) || !finite3(c->up) || !std::isfinite(c->vfov_deg))
    return fail(CLOUD_E_INVALID, "camera values must be finite");
  if (!(c->vfov_deg > 0.0f && c->vfov_deg < 180.0f))
    return fail(CLOUD_E_INVALID, "vfov_deg must be in (0, 180)");
  double f[3], r[3], u[3];
  for (int k = 0; k < 3; ++k) f[k] = (double)c->target[k] - c->pos[k];
  double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  if (!(fl > 0.0)) return fail(CLOUD_E_INVALID, "camera target equals its position");
  for (double& x : f) x /= fl;
  const double up[3] = {c->up[0], c->up[1], c->up[2]};
  r[0] = f[1] * up[2] - f[2] * up[1];
  r[1] = f[2] * up[0] - f[0] * up[2];
  r[2] = f[0] * up[1] - f[1] * up[0];
  const double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  if (!(rl > 1e-12)) return fail(CLOUD_E_INVALID, "camera up is parallel to the view direction");
  for (double& x : r) x /= rl;
  u[0] = r[1] * f[2] - r[2] * f[1];
  u[1] = r[2] * f[0] - r[0] * f[2];
  u[2] = r[0] * f[1] - r[1] * f[0];
  DevCamera d;
  for (int k = 0; k < 3; ++k) {
    d.pos[k] = c->pos[k];
    d.fwd[k] = (float)f[k];
    d.right[k] = (float)r[k];
    d.up[k] = (float)u[k];
  }
  d.tan_half = (float)std::tan((double)c->vfov_deg * M_PI / 360.0);
  d.aspect = (float)((double)W / (double)H);
  *out = d;
  return CLOUD_OK;
}

}  // namespace cloud

using namespace cloud;

#define CLOUD_GUARD_BEGIN try {
#define CLOUD_GUARD_END                                                          \
  }                                                                              \
  catch (const std::bad_alloc&) {                                                \
    return fail(CLOUD_E_NOMEM, "host allocation failed");                        \
  }                                                                              \
  catch (...) {                                                                  \
    return fail(CLOUD_E_INVALID, "internal error");                              \
  }

extern "C" {

const char* cloud_last_error(void) { return g_last_error.c_str(); }

int cloud_abi_version(void) { return CLOUD_ABI_VERSION; }

static int render_impl(const cloud_volume* volume, const cloud_camera* cameras, int32_t n_views,
                       const cloud_params* params, uint32_t frame_index, int32_t width,
                       int32_t height, float* out_rgba, uint64_t* counts, uint32_t* trace,
                       float* depth, void* hip_stream) {
  clear_error();
  if (!cameras) return fail(CLOUD_E_INVALID, "cameras is NULL");
  if (n_views < 1) return fail(CLOUD_E_INVALID, "n_views must be >= 1");
  int rc = check_image(width, height, n_views);
  if (rc) return rc;
  DevVolume v;
  int dtype;
  if ((rc = prepare_volume(volume, &v, &dtype))) return rc;
  DevParams p;
  if ((rc = prepare_params(params, volume, &p))) return rc;
  const size_t px = (size_t)width * height;
  if (counts || trace) {
    if (counts) {
      if (reinterpret_cast<uintptr_t>(counts) % 8)
        return fail(CLOUD_E_INVALID, "out_count must be 8-byte aligned");
      if ((rc = check_span(counts, 8, "out_count"))) return rc;
    }
    if (trace) {
      if (params->steps > 32) return fail(CLOUD_E_INVALID, "a lookup trace needs steps <= 32");
      if (reinterpret_cast<uintptr_t>(trace) % 8)
        return fail(CLOUD_E_INVALID, "out_trace must be 8-byte aligned");
      if ((rc = check_span(trace, px * 8 * (size_t)n_views, "out_trace"))) return rc;
    }
  } else {
    if (reinterpret_cast<uintptr_t>(out_rgba) % 16)
      return fail(CLOUD_E_INVALID, "out_rgba must be 16-byte aligned");
    if ((rc = check_span(out_rgba, px * 16 * (size_t)n_views, "out_rgba"))) return rc;
    if (depth) {
      if (reinterpret_cast<uintptr_t>(depth) % 4)
        return fail(CLOUD_E_INVALID, "out_depth must be 4-byte aligned");
      if ((rc = check_span(depth, px * 4 * (size_t)n_views, "out_depth"))) return rc;
      const uintptr_t a = reinterpret_cast<uintptr_t>(out_rgba), b = reinterpret_cast<uintptr_t>(depth);
      const size_t na = px * 16 * (size_t)n_views, nb = px * 4 * (size_t)n_views;
      if (a < b + nb && b < a + na) return fail(CLOUD_E_INVALID, "out_depth overlaps out_rgba");
    }
  }
  DevCameras cams;
  for (int i = 0; i < n_views; ++i) {
    if ((rc = prepare_camera(&cameras[i], width, height, &cams.c[i % kMaxViews]))) return rc;
    const bool last = i + 1 == n_views;
    if ((i + 1) % kMaxViews == 0 || last) {
      const int first = i - i % kMaxViews;
      const int count = i - first + 1;
      const bool image = !counts && !trace;
      hipError_t e = launch_render(v, dtype, volume->layout, p, cams, count, frame_index, width,
                                   height, image ? out_rgba + (size_t)first * px * 4 : nullptr,
                                   reinterpret_cast<unsigned long long*>(counts),
                                   trace ? trace + (size_t)first * px * 2 : nullptr,
                                   image && depth ? depth + (size_t)first * px : nullptr,
                                   static_cast<hipStream_t>(hip_stream));
      if (e != hipSuccess) return fail(CLOUD_E_HIP, std::string("render launch: ") + hipGetErrorString(e));
    }
  }
  return CLOUD_OK;
}

int cloud_render_views(const cloud_volume* volume, const cloud_camera* cameras, int32_t n_views,
                       const cloud_params* params, uint32_t frame_index, int32_t width,
                       int32_t height, float* out_rgba, void* hip_stream) {
  CLOUD_GUARD_BEGIN
  return render_impl(volume, cameras, n_views, params, frame_index, width, height, out_rgba,
                     nullptr, nullptr, nullptr, hip_stream);
  CLOUD_GUARD_END
}

int cloud_count_lookups(const cloud_volume* volume, const cloud_camera* camera,
                        const cloud_params* params, uint32_t frame_index, int32_t width,
                        int32_t height, uint64_t* out_count, void* hip_stream) {
  CLOUD_GUARD_BEGIN
  if (!out_count) return fail(CLOUD_E_INVALID, "out_count is NULL");
  return render_impl(volume, camera, 1, params, frame_index, width, height, nullptr, out_count,
                     nullptr, nullptr, hip_stream);
  CLOUD_GUARD_END
}

int cloud_lookup_trace(const cloud_volume* volume, const cloud_camera* cameras, int32_t n_views,
                       const cloud_params* params, uint32_t frame_index, int32_t width,
                       int32_t height, uint32_t* out_trace, void* hip_stream) {
  CLOUD_GUARD_BEGIN
  if (!out_trace) return fail(CLOUD_E_INVALID, "out_trace is NULL");
  if (!params) return fail(CLOUD_E_INVALID, "params is NULL");
  return render_impl(volume, cameras, n_views, params, frame_index, width, height, nullptr,
                     nullptr, out_trace, nullptr, hip_stream);
  CLOUD_GUARD_END
}

// Wavefronts of a render of n_views W x H views: four per 16x16 tile.
static size_t render_waves(int W, int H, int n_views) {
  return (size_t)((W + 15) / 16) * ((H + 15) / 16) * 4 * (size_t)n_views;
}

static int check_replay_volume(const cloud_volume* volume, DevVolume* v, int* dtype) {
  if (!volume) return fail(CLOUD_E_INVALID, "volume is NULL");
  if (volume->detail) return fail(CLOUD_E_INVALID, "the gather replay takes no detail volume");
  int rc = prepare_volume(volume, v, dtype);
  if (rc) return rc;
  if (v->nx > 1024 || v->ny > 1024 || v->nz > 1024)
    return fail(CLOUD_E_INVALID, "the gather replay codes corners of at most 1024 texels per axis");
  return CLOUD_OK;
}

static int check_codes(const uint32_t* codes, const uint32_t* slot_counts, int max_slots,
                       size_t waves) {
  if (max_slots < 1) return fail(CLOUD_E_INVALID, "max_slots must be >= 1");
  if (reinterpret_cast<uintptr_t>(codes) % 4 || reinterpret_cast<uintptr_t>(slot_counts) % 4)
    return fail(CLOUD_E_INVALID, "codes and slot_counts must be 4-byte aligned");
  int rc = check_span(codes, waves * (size_t)max_slots * 256, "codes");
  if (rc) return rc;
  return check_span(slot_counts, waves * 4, "slot_counts");
}

int cloud_gather_record(const cloud_volume* volume, const cloud_camera* cameras, int32_t n_views,
                        const cloud_params* params, uint32_t frame_index, int32_t width,
                        int32_t height, const uint32_t* trace, int32_t max_slots, uint32_t* codes,
                        uint32_t* slot_counts, void* hip_stream) {
  CLOUD_GUARD_BEGIN
  clear_error();
  if (!cameras) return fail(CLOUD_E_INVALID, "cameras is NULL");
  if (n_views < 1) return fail(CLOUD_E_INVALID, "n_views must be >= 1");
  int rc = check_image(width, height, n_views);
  if (rc) return rc;
  DevVolume v;
  int dtype;
  if ((rc = check_replay_volume(volume, &v, &dtype))) return rc;
  DevParams p;
  if ((rc = prepare_params(params, volume, &p))) return rc;
  if (params->steps > 32) return fail(CLOUD_E_INVALID, "a lookup trace needs steps <= 32");
  if ((long long)max_slots < (long long)params->steps * (1 + params->light_steps))
    return fail(CLOUD_E_INVALID, "max_slots must be >= steps * (1 + light_steps)");
  const size_t px = (size_t)width * height;
  if (reinterpret_cast<uintptr_t>(trace) % 8) return fail(CLOUD_E_INVALID, "trace must be 8-byte aligned");
  if ((rc = check_span(trace, px * 8 * (size_t)n_views, "trace"))) return rc;
  if ((rc = check_codes(codes, slot_counts, max_slots, render_waves(width, height, n_views))))
    return rc;
  const size_t view_waves = render_waves(width, height, 1);
  DevCameras cams;
  for (int i = 0; i < n_views; ++i) {
    if ((rc = prepare_camera(&cameras[i], width, height, &cams.c[i % kMaxViews]))) return rc;
    if ((i + 1) % kMaxViews == 0 || i + 1 == n_views) {
      const int first = i - i % kMaxViews;
      hipError_t e = launch_gather_record(
          v, volume->layout, p, cams, i - first + 1, frame_index, width, height,
          trace + (size_t)first * px * 2, max_slots,
          codes + (size_t)first * view_waves * (size_t)max_slots * 64,
          slot_counts + (size_t)first * view_waves, static_cast<hipStream_t>(hip_stream));
      if (e != hipSuccess) return fail(CLOUD_E_HIP, std::string("record launch: ") + hipGetErrorString(e));
    }
  }
  return CLOUD_OK;
  CLOUD_GUARD_END
}

int cloud_gather_replay(const cloud_volume* volume, int32_t n_views, int32_t width, int32_t height,
                        const uint32_t* codes, int32_t max_slots, const uint32_t* slot_counts,
                        int32_t mode, int32_t blocks_per_cu, uint32_t* out, void* hip_stream) {
  CLOUD_GUARD_BEGIN
  clear_error();
  if (n_views < 1) return fail(CLOUD_E_INVALID, "n_views must be >= 1");
  if (mode != 0 && mode != 1) return fail(CLOUD_E_INVALID, "mode must be 0 or 1");
  if (blocks_per_cu < 0 || blocks_per_cu > 64)
    return fail(CLOUD_E_INVALID, "blocks_per_cu must be in [0, 64]");
  int rc = check_image(width, height, n_views);
  if (rc) return rc;
  DevVolume v;
  int dtype;
  if ((rc = check_replay_volume(volume, &v, &dtype))) return rc;
  const size_t waves = render_waves(width, height, n_views);
  if (waves / 4 > 0x7FFFFFFF) return fail(CLOUD_E_INVALID, "too many tiles for one launch");
  if ((rc = check_codes(codes, slot_counts, max_slots, waves))) return rc;
  if (reinterpret_cast<uintptr_t>(out) % 4) return fail(CLOUD_E_INVALID, "out must be 4-byte aligned");
  if ((rc = check_span(out, waves * 64 * 4, "out"))) return rc;
  // the replay addresses the stored base through a 32-bit buffer range
  size_t bytes = 0;
  if ((rc = volume_layout_bytes(volume, volume->layout, &bytes))) return rc;
  if (bytes > 0xFFFFFF00ull)
    return fail(CLOUD_E_INVALID, "the gather replay needs a stored volume below 4 GiB");
  hipError_t e = launch_gather_replay(v, dtype, volume->layout, (uint32_t)((bytes + 15) & ~15ull),
                                      (int)(waves / 4), max_slots, codes, slot_counts, mode == 1,
                                      blocks_per_cu, out, static_cast<hipStream_t>(hip_stream));
  if (e == hipErrorInvalidValue)
    return fail(CLOUD_E_INVALID, "blocks_per_cu cannot be reached on this device");
  if (e != hipSuccess) return fail(CLOUD_E_HIP, std::string("replay launch: ") + hipGetErrorString(e));
  return CLOUD_OK;
  CLOUD_GUARD_END
}

// Bytes of a packed copy: the base in `layout`, then (256-byte aligned) the
// detail in its oct-wrap form, if the volume has one.
static int packed_bytes(const cloud_volume* dense, int layout, size_t* base_bytes, size_t* total) {
  int rc = volume_layout_bytes(dense, layout, base_bytes);
  if (rc) return rc;
  *total = *base_bytes;
  if (dense->detail) {
    const size_t dt = (size_t)dense->dnx * dense->dny * dense->dnz;
    *total = ((*base_bytes + 255) & ~(size_t)255) + dt * 8 * dtype_size(dense->dtype);
  }
  return CLOUD_OK;
}

int cloud_volume_packed_bytes(const cloud_volume* dense, int32_t layout, uint64_t* bytes) {
  CLOUD_GUARD_BEGIN
  clear_error();
  if (!bytes) return fail(CLOUD_E_INVALID, "bytes is NULL");
  if (!dense) return fail(CLOUD_E_INVALID, "volume is NULL");
  size_t b = 0, total = 0;
  const int rc = packed_bytes(dense, layout, &b, &total);
  if (rc) return rc;
  *bytes = layout == CLOUD_LAYOUT_DENSE ? b : total;
  return CLOUD_OK;
  CLOUD_GUARD_END
}

int cloud_volume_pack(const cloud_volume* dense, int32_t layout, void* dst, uint64_t dst_bytes,
                      cloud_volume* packed, void* hip_stream) {
  CLOUD_GUARD_BEGIN
  clear_error();
  if (!dense) return fail(CLOUD_E_INVALID, "volume is NULL");
  if (!packed) return fail(CLOUD_E_INVALID, "packed is NULL");
  if (dense->layout != CLOUD_LAYOUT_DENSE) return fail(CLOUD_E_INVALID, "source volume must be dense");
  if (layout != CLOUD_LAYOUT_QUAD && layout != CLOUD_LAYOUT_OCT)
    return fail(CLOUD_E_INVALID, "target layout must be quad (1) or oct (2)");
  DevVolume v;
  int dtype, rc;
  if ((rc = prepare_volume(dense, &v, &dtype))) return rc;
  size_t base_bytes = 0, need = 0;
  if ((rc = packed_bytes(dense, layout, &base_bytes, &need))) return rc;
  if (dst_bytes < need) return fail(CLOUD_E_INVALID, "dst is smaller than the packed volume");
  if (reinterpret_cast<uintptr_t>(dst) % 16) return fail(CLOUD_E_INVALID, "dst must be 16-byte aligned");
  if ((rc = check_span(dst, need, "dst"))) return rc;
  const char* d0 = static_cast<const char*>(dst);
  const size_t es = dtype_size(dtype);
  const char* s0 = static_cast<const char*>(dense->base);
  const size_t sbytes = (size_t)dense->nx * dense->ny * dense->nz * es;
  if (d0 < s0 + sbytes && s0 < d0 + need) return fail(CLOUD_E_INVALID, "dst overlaps the volume");
  if (dense->detail) {
    const char* t0 = static_cast<const char*>(dense->detail);
    const size_t tbytes = (size_t)dense->dnx * dense->dny * dense->dnz * es;
    if (d0 < t0 + tbytes && t0 < d0 + need) return fail(CLOUD_E_INVALID, "dst overlaps the detail volume");
  }
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  int brick[3];
  brick_shape(dense, brick);   // validated by packed_bytes
  hipError_t e = launch_pack(dense->base, (int)es, dense->nx, dense->ny, dense->nz, layout, brick,
                             dst, s);
  if (e != hipSuccess) return fail(CLOUD_E_HIP, std::string("pack launch: ") + hipGetErrorString(e));
  void* ddst = nullptr;
  if (dense->detail) {
    ddst = static_cast<char*>(dst) + ((base_bytes + 255) & ~(size_t)255);
    e = launch_pack_detail(dense->detail, (int)es, dense->dnx, dense->dny, dense->dnz, ddst, s);
    if (e != hipSuccess) return fail(CLOUD_E_HIP, std::string("pack launch: ") + hipGetErrorString(e));
  }
  *packed = *dense;
  packed->base = dst;
  packed->layout = layout;
  for (int k = 0; k < 3; ++k) packed->brick_log2[k] = brick[k];
  if (dense->detail) packed->detail = ddst;
  return CLOUD_OK;
  CLOUD_GUARD_END
}

int cloud_render(const cloud_volume* volume, const cloud_camera* camera,
                 const cloud_params* params, uint32_t frame_index, int32_t width, int32_t height,
                 float* out_rgba, void* hip_stream) {
  if (!camera) return fail(CLOUD_E_INVALID, "camera is NULL");
  return cloud_render_views(volume, camera, 1, params, frame_index, width, height, out_rgba,
                            hip_stream);
}

int cloud_march_rays(const cloud_volume* volume, const float* origins, const float* dirs,
                     const uint32_t* pixel_xy, int64_t n, const cloud_params* params,
                     uint32_t frame_index, float* out_rgba, void* hip_stream) {
  CLOUD_GUARD_BEGIN
  clear_error();
  if (n < 0) return fail(CLOUD_E_INVALID, "n must be >= 0");
  if (n > (int64_t)1 << 31) return fail(CLOUD_E_INVALID, "n must be <= 2^31");
  DevVolume v;
  int dtype, rc;
  if ((rc = prepare_volume(volume, &v, &dtype))) return rc;
  DevParams p;
  if ((rc = prepare_params(params, volume, &p))) return rc;
  if (n == 0) return CLOUD_OK;
  if ((rc = check_span(origins, (size_t)n * 12, "origins"))) return rc;
  if ((rc = check_span(dirs, (size_t)n * 12, "dirs"))) return rc;
  if (pixel_xy && (rc = check_span(pixel_xy, (size_t)n * 8, "pixel_xy"))) return rc;
  if (reinterpret_cast<uintptr_t>(out_rgba) % 16)
    return fail(CLOUD_E_INVALID, "out_rgba must be 16-byte aligned");
  if ((rc = check_span(out_rgba, (size_t)n * 16, "out_rgba"))) return rc;
  hipError_t e = launch_rays(v, dtype, volume->layout, p, frame_index, origins, dirs, pixel_xy, n,
                             out_rgba,
                             static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(CLOUD_E_HIP, std::string("march launch: ") + hipGetErrorString(e));
  return CLOUD_OK;
  CLOUD_GUARD_END
}

// The checks of a resolve of n_views images current against history into
// out; *copy receives whether it is a copy (no history, or frame 0).
static int check_resolve(const float* current, const float* history, const float* out,
                         int32_t width, int32_t height, int32_t n_views, float blend,
                         uint32_t frame_index, bool* copy) {
  int rc = check_image(width, height, n_views);
  if (rc) return rc;
  if (!std::isfinite(blend) || !(blend > 0.0f) || blend > 1.0f)
    return fail(CLOUD_E_INVALID, "blend must be in (0, 1]");
  const size_t bytes = (size_t)width * height * 16 * (size_t)n_views;
  if ((rc = check_span(current, bytes, "current"))) return rc;
  if ((rc = check_span(out, bytes, "out"))) return rc;
  *copy = history == nullptr || frame_index == 0;
  if (!*copy && (rc = check_span(history, bytes, "history"))) return rc;
  const uintptr_t a = reinterpret_cast<uintptr_t>(current), b = reinterpret_cast<uintptr_t>(out);
  if ((a | b | reinterpret_cast<uintptr_t>(history)) % 16)
    return fail(CLOUD_E_INVALID, "images must be 16-byte aligned");
  if (a < b + bytes && b < a + bytes) return fail(CLOUD_E_INVALID, "out overlaps current");
  if (!*copy && history != out) {
    const uintptr_t h = reinterpret_cast<uintptr_t>(history);
    if (h < b + bytes && b < h + bytes)
      return fail(CLOUD_E_INVALID, "out partially overlaps history");
  }
  return CLOUD_OK;
}

int cloud_taa_resolve(const float* current, const float* history, float* out, int32_t width,
                      int32_t height, float blend, uint32_t frame_index, void* hip_stream) {
  CLOUD_GUARD_BEGIN
  clear_error();
  bool copy = false;
  int rc = check_resolve(current, history, out, width, height, 1, blend, frame_index, &copy);
  if (rc) return rc;
  hipError_t e = launch_taa(current, history, out, width, height, blend, copy,
                            static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(CLOUD_E_HIP, std::string("resolve launch: ") + hipGetErrorString(e));
  return CLOUD_OK;
  CLOUD_GUARD_END
}

int cloud_render_resolve(const cloud_volume* volume, const cloud_camera* cameras,
                         int32_t n_views, const cloud_params* params, uint32_t frame_index,
                         int32_t width, int32_t height, float* out_rgba, const float* prev_rgba,
                         const float* history, float* resolved, float blend,
                         uint32_t prev_frame_index, void* hip_stream) {
  CLOUD_GUARD_BEGIN
  clear_error();
  if (!cameras) return fail(CLOUD_E_INVALID, "cameras is NULL");
  if (n_views < 1) return fail(CLOUD_E_INVALID, "n_views must be >= 1");
  int rc = check_image(width, height, n_views);
  if (rc) return rc;
  DevVolume v;
  int dtype;
  if ((rc = prepare_volume(volume, &v, &dtype))) return rc;
  DevParams p;
  if ((rc = prepare_params(params, volume, &p))) return rc;
  const size_t px = (size_t)width * height, bytes = px * 16 * (size_t)n_views;
  if (reinterpret_cast<uintptr_t>(out_rgba) % 16)
    return fail(CLOUD_E_INVALID, "out_rgba must be 16-byte aligned");
  if ((rc = check_span(out_rgba, bytes, "out_rgba"))) return rc;
  bool copy = false;
  if ((rc = check_resolve(prev_rgba, history, resolved, width, height, n_views, blend,
                          prev_frame_index, &copy)))
    return rc;
  // the render runs beside the resolve: its output must be none of the
  // resolve's images
  const uintptr_t o = reinterpret_cast<uintptr_t>(out_rgba);
  const float* others[3] = {prev_rgba, resolved, copy ? nullptr : history};
  for (const float* q : others) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(q);
    if (q && a < o + bytes && o < a + bytes)
      return fail(CLOUD_E_INVALID, "out_rgba overlaps prev_rgba, history or resolved");
  }
  DevCameras cams;
  for (int i = 0; i < n_views; ++i) {
    if ((rc = prepare_camera(&cameras[i], width, height, &cams.c[i % kMaxViews]))) return rc;
    if ((i + 1) % kMaxViews == 0 || i + 1 == n_views) {
      const int first = i - i % kMaxViews;
      const size_t off = (size_t)first * px * 4;
      hipError_t e = launch_render_resolve(
          v, dtype, volume->layout, p, cams, i - first + 1, frame_index, width, height,
          out_rgba + off, prev_rgba + off, copy ? nullptr : history + off, resolved + off, blend,
          copy, static_cast<hipStream_t>(hip_stream));
      if (e != hipSuccess)
        return fail(CLOUD_E_HIP, std::string("render and resolve launch: ") + hipGetErrorString(e));
    }
  }
  return CLOUD_OK;
  CLOUD_GUARD_END
}

int cloud_render_depth(const cloud_volume* volume, const cloud_camera* camera,
                       const cloud_params* params, uint32_t frame_index, int32_t width,
                       int32_t height, float* out_rgba, float* out_depth, void* hip_stream) {
  CLOUD_GUARD_BEGIN
  if (!out_depth) return fail(CLOUD_E_INVALID, "out_depth is NULL");
  return render_impl(volume, camera, 1, params, frame_index, width, height, out_rgba, nullptr,
                     nullptr, out_depth, hip_stream);
  CLOUD_GUARD_END
}

int cloud_taa_resolve_reproject(const float* current, const float* depth, const float* history,
                                float* out, const cloud_camera* camera,
                                const cloud_camera* prev_camera, int32_t width, int32_t height,
                                float blend, uint32_t frame_index, void* hip_stream) {
  CLOUD_GUARD_BEGIN
  clear_error();
  int rc = check_image(width, height, 1);
  if (rc) return rc;
  if (!std::isfinite(blend) || !(blend > 0.0f) || blend > 1.0f)
    return fail(CLOUD_E_INVALID, "blend must be in (0, 1]");
  const size_t bytes = (size_t)width * height * 16;
  if ((rc = check_span(current, bytes, "current"))) return rc;
  if ((rc = check_span(out, bytes, "out"))) return rc;
  const uintptr_t a = reinterpret_cast<uintptr_t>(current), b = reinterpret_cast<uintptr_t>(out);
  if ((a | b | reinterpret_cast<uintptr_t>(history)) % 16)
    return fail(CLOUD_E_INVALID, "images must be 16-byte aligned");
  if (a < b + bytes && b < a + bytes) return fail(CLOUD_E_INVALID, "out overlaps current");
  const bool copy = history == nullptr || frame_index == 0;
  if (copy) {
    hipError_t e = launch_taa(current, nullptr, out, width, height, blend, true,
                              static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(CLOUD_E_HIP, std::string("resolve launch: ") + hipGetErrorString(e));
    return CLOUD_OK;
  }
  if ((rc = check_span(history, bytes, "history"))) return rc;
  if ((rc = check_span(depth, bytes / 4, "depth"))) return rc;
  if (reinterpret_cast<uintptr_t>(depth) % 4) return fail(CLOUD_E_INVALID, "depth must be 4-byte aligned");
  const uintptr_t h = reinterpret_cast<uintptr_t>(history), dp = reinterpret_cast<uintptr_t>(depth);
  if (h < b + bytes && b < h + bytes)
    return fail(CLOUD_E_INVALID, "out overlaps history (a reprojected resolve cannot run in place)");
  if (dp < b + bytes && b < dp + bytes / 4) return fail(CLOUD_E_INVALID, "out overlaps depth");
  DevCamera cam, prev;
  if ((rc = prepare_camera(camera, width, height, &cam))) return rc;
  if ((rc = prepare_camera(prev_camera, width, height, &prev))) return rc;
  hipError_t e = launch_taa_reproject(current, depth, history, out, cam, prev, width, height, blend,
                                      static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(CLOUD_E_HIP, std::string("resolve launch: ") + hipGetErrorString(e));
  return CLOUD_OK;
  CLOUD_GUARD_END
}

int cloud_composite(const float* cloud, int32_t cloud_width, int32_t cloud_height,
                    const float* background, float* out, int32_t width, int32_t height,
                    void* hip_stream) {
  CLOUD_GUARD_BEGIN
  clear_error();
  int rc = check_image(width, height, 1);
  if (rc) return rc;
  if ((rc = check_image(cloud_width, cloud_height, 1))) return rc;
  const size_t lbytes = (size_t)cloud_width * cloud_height * 16, bytes = (size_t)width * height * 16;
  if ((rc = check_span(cloud, lbytes, "cloud"))) return rc;
  if ((rc = check_span(background, bytes, "background"))) return rc;
  if ((rc = check_span(out, bytes, "out"))) return rc;
  const uintptr_t c = reinterpret_cast<uintptr_t>(cloud), b = reinterpret_cast<uintptr_t>(background),
                  o = reinterpret_cast<uintptr_t>(out);
  if ((c | b | o) % 16) return fail(CLOUD_E_INVALID, "images must be 16-byte aligned");
  if (c < o + bytes && o < c + lbytes) return fail(CLOUD_E_INVALID, "out overlaps cloud");
  if (b != o && b < o + bytes && o < b + bytes)
    return fail(CLOUD_E_INVALID, "out partially overlaps background");
  hipError_t e = launch_composite(cloud, cloud_width, cloud_height, background, out, width, height,
                                  static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(CLOUD_E_HIP, std::string("composite launch: ") + hipGetErrorString(e));
  return CLOUD_OK;
  CLOUD_GUARD_END
}

int cloud_volume_occupancy_bytes(const cloud_volume* dense, uint64_t* bytes, int32_t* log2_brick) {
  CLOUD_GUARD_BEGIN
  clear_error();
  if (!bytes || !log2_brick) return fail(CLOUD_E_INVALID, "NULL output");
  size_t b = 0;
  const int rc = volume_layout_bytes(dense, CLOUD_LAYOUT_DENSE, &b);
  if (rc) return rc;
  const int lg = occupancy_log2(dense);
  int nbx, nby, nbz;
  occupancy_dims(dense, lg, &nbx, &nby, &nbz);
  *bytes = (uint64_t)occupancy_words(nbx, nby, nbz) * 4;
  *log2_brick = lg;
  return CLOUD_OK;
  CLOUD_GUARD_END
}

int cloud_volume_occupancy(const cloud_volume* dense, uint32_t* dst, uint64_t dst_bytes,
                           cloud_volume* with_occupancy, void* hip_stream) {
  CLOUD_GUARD_BEGIN
  clear_error();
  if (!dense) return fail(CLOUD_E_INVALID, "volume is NULL");
  if (!with_occupancy) return fail(CLOUD_E_INVALID, "with_occupancy is NULL");
  if (dense->layout != CLOUD_LAYOUT_DENSE) return fail(CLOUD_E_INVALID, "source volume must be dense");
  cloud_volume src = *dense;
  src.occupancy = nullptr;   // the source's own bitmap (if any) is not needed
  DevVolume v;
  int dtype, rc;
  if ((rc = prepare_volume(&src, &v, &dtype))) return rc;
  const int lg = occupancy_log2(dense);
  int nbx, nby, nbz;
  occupancy_dims(dense, lg, &nbx, &nby, &nbz);
  const size_t need = (size_t)occupancy_words(nbx, nby, nbz) * 4;
  if (dst_bytes < need) return fail(CLOUD_E_INVALID, "dst is smaller than the bitmap");
  if (reinterpret_cast<uintptr_t>(dst) % 4) return fail(CLOUD_E_INVALID, "dst must be 4-byte aligned");
  if ((rc = check_span(dst, need, "dst"))) return rc;
  hipError_t e = launch_occupancy(dense->base, (int)dtype_size(dtype), dense->nx, dense->ny,
                                  dense->nz, lg, nbx, nby, nbz, dst,
                                  static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(CLOUD_E_HIP, std::string("occupancy launch: ") + hipGetErrorString(e));
  *with_occupancy = *dense;
  with_occupancy->occupancy = dst;
  with_occupancy->occupancy_log2 = lg;
  return CLOUD_OK;
  CLOUD_GUARD_END
}

int cloud_tune(const char* key, int32_t value) {
  CLOUD_GUARD_BEGIN
  clear_error();
  if (!key) return fail(CLOUD_E_INVALID, "key is NULL");
  const std::string k(key);
  if (k == "supertile") {
    if (value < -1 || value > 64) return fail(CLOUD_E_INVALID, "supertile must be in [-1, 64]");
    tuning().supertile = value;
    return CLOUD_OK;
  }
  if (k == "xcd_run") {
    if (value < -1 || value > 65536) return fail(CLOUD_E_INVALID, "xcd_run must be in [-1, 65536]");
    tuning().xcd_run = value;
    return CLOUD_OK;
  }
  if (k == "taa_tile") {
    if (value != 16 && value != 32 && value != 64)
      return fail(CLOUD_E_INVALID, "taa_tile must be 16, 32 or 64");
    tuning().taa_tile = value;
    return CLOUD_OK;
  }
  if (k == "render_blocks_per_cu") {
    if (value < 0 || value > 64) return fail(CLOUD_E_INVALID, "render_blocks_per_cu must be in [0, 64]");
    if (value > 0 && residency_lds(value, 4096) < 0)
      return fail(CLOUD_E_INVALID, "render_blocks_per_cu: this cap cannot be set through LDS");
    tuning().render_blocks_per_cu = value;
    return CLOUD_OK;
  }
  if (k == "serve_blocks_per_cu") {
    if (value < 0 || value > 64) return fail(CLOUD_E_INVALID, "serve_blocks_per_cu must be in [0, 64]");
    tuning().serve_blocks_per_cu = value;
    return CLOUD_OK;
  }
  return fail(CLOUD_E_INVALID, "unknown tuning key " + k);
  CLOUD_GUARD_END
}

int cloud_check_buffer(const void* ptr, uint64_t bytes) {
  CLOUD_GUARD_BEGIN
  clear_error();
  return check_span(ptr, (size_t)bytes, "buffer");
  CLOUD_GUARD_END
}

int cloud_jitter_offsets(const uint32_t* pixel_xy, int64_t n, uint32_t frame_index, uint32_t seed,
                         uint32_t* out_bits, void* hip_stream) {
  CLOUD_GUARD_BEGIN
  clear_error();
  if (n < 0 || n > (int64_t)1 << 31) return fail(CLOUD_E_INVALID, "n must be in [0, 2^31]");
  if (n == 0) return CLOUD_OK;
  int rc;
  if ((rc = check_span(pixel_xy, (size_t)n * 8, "pixel_xy"))) return rc;
  if ((rc = check_span(out_bits, (size_t)n * 4, "out_bits"))) return rc;
  hipError_t e = launch_jitter(pixel_xy, n, frame_index, seed, out_bits,
                               static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(CLOUD_E_HIP, std::string("jitter launch: ") + hipGetErrorString(e));
  return CLOUD_OK;
  CLOUD_GUARD_END
}

}  // extern "C"

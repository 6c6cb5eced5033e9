// C ABI of the library (declared in include/rgx.h): argument checking,
// device-memory ownership of the acceleration structure and the launch
// descriptors.  All device work is enqueued on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/rgx.h"
#include "common.hpp"
#include "internal.hpp"

using namespace rgx;

static_assert(RGX_STAT_Q == ST_Q && RGX_STAT_P == ST_P && RGX_STAT_SAMPLES == ST_SAMPLES &&
                  RGX_STAT_SEGMENTS == ST_SEGMENTS && RGX_STAT_CLOSEST == ST_CLOSEST &&
                  RGX_STAT_BOX_ONLY == ST_BOX_ONLY && RGX_STAT_NODES == ST_NODES &&
                  RGX_STAT_LEAVES == ST_LEAVES && RGX_STAT_WINDOWS == ST_WINDOWS &&
                  RGX_STAT_CHUNKED == ST_CHUNKED && RGX_STAT_KCYC_TILE == ST_KCYC_TILE &&
                  RGX_STAT_T_END == ST_T_END &&
                  RGX_NSTAT == kNStat,
              "stat slots");
static_assert(RGX_MAX_GAUSSIANS == RGX_MAX_GAUSSIANS_INTERNAL, "size limit");

namespace {

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct rgx_context {
  int device = 0;
  int n_cu = 256;
  std::string last_error;
  int32_t *queue = nullptr;        // 8 persistent-launch queues + error flag
  std::map<std::tuple<int, int, int, int>, int32_t *> tile_orders;
  // optional per-launch timing: event pairs recorded on the caller's stream
  bool timing = false;
  std::vector<hipEvent_t> ev;       // 2 per recorded launch, reused after a reset
  std::vector<int> ev_kind;         // RGX_KERN_* of each recorded launch
  size_t ev_used = 0;
  double *partial = nullptr;        // per-block partial sums of rgx_isotropic_loss
  int64_t partial_cap = 0;
  uint64_t build_serial = 0;        // bumped by every build on the context: names a structure build
  int32_t replayed = 0;             // whether the last backward replayed
  double *iso_scratch = nullptr;    // device address of the fixed loss workspace on this device
  int64_t record_limit = 0;         // cap on a forward state's record pool in bytes (0: none)
};

// Records hipEvents on `stream` around `launch` when timing is enabled.
template <class F>
static hipError_t timed(rgx_context *ctx, int kind, hipStream_t stream, F &&launch) {
  if (!ctx->timing) return launch();
  if (ctx->ev_used + 2 > ctx->ev.size()) {
    for (int k = 0; k < 2; k++) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      ctx->ev.push_back(e);
    }
    ctx->ev_kind.resize(ctx->ev.size() / 2);
  }
  const size_t i = ctx->ev_used;
  hipError_t r = hipEventRecord(ctx->ev[i], stream);
  if (r == hipSuccess) r = launch();
  if (r == hipSuccess) r = hipEventRecord(ctx->ev[i + 1], stream);
  if (r == hipSuccess) {
    ctx->ev_kind[i / 2] = kind;
    ctx->ev_used += 2;
  }
  return r;
}

struct rgx_bvh {
  rgx_context *ctx = nullptr;
  int64_t n = 0, cap = 0;
  int32_t sh_degree = 0, sh_k = 1, col_stride = 4, col_cap = 0;
  int32_t n_sg = 0;                 // spherical-Gaussian lobes per Gaussian
  float sigma_eps = 0.01f;
  int morton_bits = 21;
  int sorted_sel = 0;
  uint64_t serial = 0;              // the context's build serial of the current contents
  DevBuf geom_user, aabb_user, aux_user, aux, active, bounds, counters, keys0, keys1, vals0, vals1, hist, geom,
      aabb, col, nodes, nodes4, seg, acc, zsum, sg_user, sgrec, sgacc;
};

// Forward state: what one forward rendered and what its searches found.
struct rgx_fwd {
  rgx_context *ctx = nullptr;       // compared only: the state may outlive its context
  int device = 0;                   // the context's device, for rgx_fwd_destroy
  const rgx_bvh *bvh = nullptr;     // compared, never dereferenced (the structure may be gone)
  uint64_t serial = 0;              // build serial the forward rendered
  int64_t n = 0;                    // Gaussians of that build
  std::vector<rgx_camera> cams;
  rgx_render_opts opts;
  int64_t rays = 0, tiles = 0;
  bool recorded = false;            // closest hits and window lists recorded
  bool has_totals = false;          // statistics totals reduced into `totals`
  DevBuf replay;                    // [rays][kReplayK] closest-hit results
  DevBuf wrec;                      // window-list pool (64-bit counter first)
  DevBuf wrec_tile;                 // per tile: (complete, first record)
  DevBuf totals;                    // int64 [RGX_NTOT]
  std::vector<void *> retired;      // outgrown buffers: a captured graph may still use them
};

static rgx_status fail(rgx_context *ctx, rgx_status s, const std::string &msg) {
  if (ctx) ctx->last_error = msg;
  return s;
}

static rgx_status hip_fail(rgx_context *ctx, hipError_t e, const char *where) {
  return fail(ctx, RGX_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr)                                  \
  do {                                                      \
    hipError_t e_ = (expr);                                 \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr);  \
  } while (0)

// Makes `device` current and clears an error left pending by earlier HIP
// calls outside the library, so that the launch checks of this call report
// only this call's own errors.
static hipError_t enter(int device) {
  (void)hipGetLastError();
  return hipSetDevice(device);
}

static hipError_t ensure(DevBuf &b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return hipSuccess;
  if (b.p) { (void)hipFree(b.p); b.p = nullptr; b.bytes = 0; }
  hipError_t e = hipMalloc(&b.p, std::max<size_t>(bytes, 256));
  if (e == hipSuccess) b.bytes = std::max<size_t>(bytes, 256);
  return e;
}

static void release(DevBuf &b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

extern "C" {

const char *rgx_status_string(rgx_status s) {
  switch (s) {
    case RGX_OK: return "ok";
    case RGX_ERR_INVALID_ARG: return "invalid argument";
    case RGX_ERR_OUT_OF_MEMORY: return "out of device memory";
    case RGX_ERR_HIP: return "HIP runtime error";
    case RGX_ERR_UNSUPPORTED: return "unsupported option";
    case RGX_ERR_STATE: return "invalid state";
  }
  return "unknown status";
}

const char *rgx_last_error(const rgx_context *ctx) { return ctx ? ctx->last_error.c_str() : ""; }

rgx_status rgx_create(int device, rgx_context **out) {
  if (!out) return RGX_ERR_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return RGX_ERR_INVALID_ARG;
  rgx_context *ctx = new rgx_context();
  ctx->device = device;
  hipError_t e = hipSetDevice(device);
  hipDeviceProp_t prop;
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, device);
  if (e == hipSuccess) {
    ctx->n_cu = prop.multiProcessorCount;
    e = hipMalloc((void **)&ctx->queue, 16 * sizeof(int32_t));
  }
  if (e == hipSuccess) e = hipMemset(ctx->queue, 0, 16 * sizeof(int32_t));
  // device address of this device's copy of the fixed workspace used by the
  // allocation-free entry point (the array's name is not a device address)
  if (e == hipSuccess) e = iso_scratch_resolve(&ctx->iso_scratch);
  if (e != hipSuccess) {
    delete ctx;
    return RGX_ERR_HIP;
  }
  *out = ctx;
  return RGX_OK;
}

int32_t rgx_backward_replayed(const rgx_context *ctx) { return ctx ? ctx->replayed : 0; }

void rgx_destroy(rgx_context *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  for (auto &kv : ctx->tile_orders) (void)hipFree(kv.second);
  if (ctx->queue) (void)hipFree(ctx->queue);
  for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
  if (ctx->partial) (void)hipFree(ctx->partial);
  delete ctx;
}

void rgx_bvh_destroy(rgx_bvh *b) {
  if (!b) return;
  DevBuf *all[] = {&b->geom_user, &b->aabb_user, &b->aux_user, &b->aux, &b->active, &b->bounds, &b->counters, &b->keys0,
                   &b->keys1, &b->vals0, &b->vals1, &b->hist, &b->geom, &b->aabb, &b->col,
                   &b->nodes, &b->nodes4, &b->seg, &b->acc, &b->zsum,
                   &b->sg_user, &b->sgrec, &b->sgacc};
  for (DevBuf *d : all) release(*d);
  delete b;
}

int64_t rgx_bvh_size(const rgx_bvh *b) { return b ? b->n : 0; }

rgx_status rgx_build_bvh(rgx_context *ctx, const rgx_gaussians *g, const rgx_build_opts *opts,
                         rgx_bvh **bvh, hipStream_t stream) {
  if (!ctx || !g || !bvh) return fail(ctx, RGX_ERR_INVALID_ARG, "null argument");
  if (g->n <= 0) return fail(ctx, RGX_ERR_INVALID_ARG, "n out of range");
  if (g->n > RGX_MAX_GAUSSIANS)
    return fail(ctx, RGX_ERR_UNSUPPORTED, "n above RGX_MAX_GAUSSIANS");
  if (g->sh_degree < 0 || g->sh_degree > 3)
    return fail(ctx, RGX_ERR_INVALID_ARG, "sh_degree must be 0..3");
  if (!g->means || !g->log_scales || !g->quats || !g->density || !g->sh)
    return fail(ctx, RGX_ERR_INVALID_ARG, "null parameter array");
  if (g->n_sg < 0 || g->n_sg > kMaxSg || (g->n_sg > 0 && !g->sg))
    return fail(ctx, RGX_ERR_INVALID_ARG, "n_sg must be 0..7, with sg given when > 0");
  const float sigma_eps = opts ? opts->sigma_eps : 0.01f;
  const int bits = (opts && opts->morton_bits) ? opts->morton_bits : 21;
  if (!(sigma_eps > 0.0f) || !std::isfinite(sigma_eps))
    return fail(ctx, RGX_ERR_INVALID_ARG, "sigma_eps must be > 0");
  if (bits < 1 || bits > 21) return fail(ctx, RGX_ERR_INVALID_ARG, "morton_bits must be 1..21");
  HIP_TRY(ctx, enter(ctx->device));
  rgx_bvh *b = *bvh;
  const bool fresh = b == nullptr;
  if (fresh) {
    b = new rgx_bvh();
    b->ctx = ctx;
  }
  const int64_t n = g->n;
  const int sh_k = (g->sh_degree + 1) * (g->sh_degree + 1);
  const int col_stride = kColFloats;   // fixed record length: the march reads it unconditionally
  const int64_t nb = (n + 4095) / 4096;
  const size_t nodes_n = (size_t)std::max<int64_t>(n - 1, 1);
  hipError_t e = hipSuccess;
#define ENS(buf, bytes) \
  if (e == hipSuccess) e = ensure(b->buf, (bytes))
  ENS(geom_user, (size_t)n * kGeomFloats * 4);
  ENS(aabb_user, (size_t)n * 6 * 4);
  ENS(aux_user, (size_t)n * kAuxFloats * 4);
  ENS(aux, (size_t)n * kAuxFloats * 4);
  ENS(active, (size_t)n);
  ENS(bounds, 64);
  ENS(counters, 64);
  ENS(keys0, (size_t)n * 8);
  ENS(keys1, (size_t)n * 8);
  ENS(vals0, (size_t)n * 4);
  ENS(vals1, (size_t)n * 4);
  ENS(hist, (size_t)nb * 256 * 4);
  ENS(geom, (size_t)n * kGeomFloats * 4);
  ENS(aabb, (size_t)n * 6 * 4);
  ENS(col, (size_t)n * col_stride * 4);
  ENS(nodes, nodes_n * 16 * 4);
  ENS(nodes4, nodes_n * kNode4Floats * 4);
  int64_t P = 1;
  while (P < n) P <<= 1;
  ENS(seg, (size_t)(2 * P) * 6 * 4);
  ENS(acc, (size_t)n * kAccFloats * 4);
  if (g->n_sg > 0) {
    ENS(sg_user, (size_t)n * kSgFloats * 4);
    ENS(sgrec, (size_t)n * kSgFloats * 4);
    ENS(sgacc, (size_t)n * kSgAccFloats * 4);
  }
#undef ENS
  if (e != hipSuccess) {
    if (fresh) rgx_bvh_destroy(b);
    return fail(ctx, e == hipErrorOutOfMemory ? RGX_ERR_OUT_OF_MEMORY : RGX_ERR_HIP,
                std::string("allocation: ") + hipGetErrorString(e));
  }
  b->n = n;
  b->serial = ++ctx->build_serial;
  b->sh_degree = g->sh_degree;
  b->sh_k = sh_k;
  b->col_stride = col_stride;
  b->sigma_eps = sigma_eps;
  b->morton_bits = bits;
  b->n_sg = g->n_sg;
  BuildArgs a;
  a.n = n;
  a.means = g->means; a.log_scales = g->log_scales; a.quats = g->quats; a.density = g->density;
  a.sh = g->sh;
  a.sg = g->sg;
  a.n_sg = g->n_sg;
  a.sg_user = (float *)b->sg_user.p;
  a.sgrec = (float *)b->sgrec.p;
  a.sh_k = sh_k; a.col_stride = col_stride; a.morton_bits = bits; a.sigma_eps = sigma_eps;
  a.geom_user = (float *)b->geom_user.p; a.aabb_user = (float *)b->aabb_user.p;
  a.aux_user = (float *)b->aux_user.p; a.aux = (float *)b->aux.p;
  a.active = (uint8_t *)b->active.p; a.bounds = (uint32_t *)b->bounds.p;
  a.counters = (int32_t *)b->counters.p;
  a.keys[0] = (uint64_t *)b->keys0.p; a.keys[1] = (uint64_t *)b->keys1.p;
  a.vals[0] = (uint32_t *)b->vals0.p; a.vals[1] = (uint32_t *)b->vals1.p;
  a.sort_hist = (uint32_t *)b->hist.p;
  a.sorted_sel = &b->sorted_sel;
  a.geom = (float *)b->geom.p; a.aabb = (float *)b->aabb.p; a.col = (float *)b->col.p;
  a.nodes = (float *)b->nodes.p; a.seg = (float *)b->seg.p;
  a.nodes4 = (float *)b->nodes4.p;
  e = timed(ctx, RGX_KERN_BUILD, stream, [&] {
    hipError_t r = launch_build(a, stream);
    if (r == hipSuccess) r = launch_fill(b->acc.p, n * kAccFloats, 0u, stream);
    if (r == hipSuccess && g->n_sg > 0) r = launch_fill(b->sgacc.p, n * kSgAccFloats, 0u, stream);
    return r;
  });
  if (e != hipSuccess) {
    if (fresh) rgx_bvh_destroy(b);
    return hip_fail(ctx, e, "build launch");
  }
  *bvh = b;
  return RGX_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Launch descriptors

static SceneDev scene_of(const rgx_bvh *b) {
  SceneDev s;
  s.geom = (const float *)b->geom.p;
  s.col = (const float *)b->col.p;
  s.nodes = (const float *)b->nodes.p;
  s.nodes4 = (const float *)b->nodes4.p;
  s.aabb = (const float *)b->aabb.p;
  s.counters = (const int32_t *)b->counters.p;
  s.perm = (const uint32_t *)(b->sorted_sel ? b->vals1.p : b->vals0.p);
  s.aux = (const float *)b->aux.p;
  s.sg = b->n_sg > 0 ? (const float *)b->sgrec.p : nullptr;
  s.n_sg = b->n_sg;
  s.n = b->n;
  return s;
}

static int ilog2(int v) {
  int r = 0;
  while ((1 << r) < v) r++;
  return r;
}

static rgx_status make_opts(rgx_context *ctx, const rgx_bvh *b, const rgx_render_opts *o,
                            MarchOpts &m) {
  if (!o) return fail(ctx, RGX_ERR_INVALID_ARG, "null opts");
  memset(&m, 0, sizeof m);
  if (!(o->n_s == 1 || o->n_s == 2 || o->n_s == 4 || o->n_s == 8 || o->n_s == 16))
    return fail(ctx, RGX_ERR_UNSUPPORTED, "n_s must be 1, 2, 4, 8 or 16");
  if (o->adaptive) {
    if (!(o->dt_min > 0.0f) || !(o->dt_max >= o->dt_min) || !(o->beta > 0.0f))
      return fail(ctx, RGX_ERR_INVALID_ARG, "adaptive needs 0 < dt_min <= dt_max and beta > 0");
  } else if (!(o->dt > 0.0f)) {
    return fail(ctx, RGX_ERR_INVALID_ARG, "dt must be > 0");
  }
  if (!(o->t_eps >= 0.0f)) return fail(ctx, RGX_ERR_INVALID_ARG, "t_eps must be >= 0");
  if (o->ess < 0 || o->ess > 2) return fail(ctx, RGX_ERR_INVALID_ARG, "ess must be 0, 1 or 2");
  int tw = o->tile_w, th = o->tile_h;
  if (tw == 0 && th == 0) { tw = 8; th = 8; }
  if (o->ray_order == 1 && !(tw * th == 64 && (tw & (tw - 1)) == 0))
    return fail(ctx, RGX_ERR_INVALID_ARG, "tile_w * tile_h must be 64 with tile_w a power of 2");
  if (o->ray_order != 0 && o->ray_order != 1)
    return fail(ctx, RGX_ERR_INVALID_ARG, "ray_order must be 0 or 1");
  m.adaptive = o->adaptive ? 1 : 0;
  m.dt = o->dt;
  m.dt_min = o->dt_min;
  m.dt_max = o->dt_max;
  m.inv_beta = o->adaptive ? 1.0f / o->beta : 0.0f;
  m.n_s = o->n_s;
  m.t_eps = o->t_eps;
  m.ess = o->ess;
  m.brute_force = o->brute_force ? 1 : 0;
  m.ray_order = o->ray_order;
  m.tile_w = tw;
  m.tile_h = th;
  m.tile_w_log2 = ilog2(tw);
  m.persistent = o->persistent ? 1 : 0;
  if (o->window_segments < 0 || o->window_segments > 64)
    return fail(ctx, RGX_ERR_INVALID_ARG, "window_segments must be 0..64");
  m.window_segments = o->window_segments ? o->window_segments : 1;
  for (int i = 0; i < 3; i++) m.bg[i] = o->bg[i];
  m.sh_k = b->sh_k;
  m.col_stride = b->col_stride;
  if (b->n_sg > 0 && m.n_s != 8)
    return fail(ctx, RGX_ERR_UNSUPPORTED, "spherical-Gaussian colour lobes need n_s = 8");
  return RGX_OK;
}

static rgx_status check_camera(rgx_context *ctx, const rgx_camera &c) {
  if (c.width <= 0 || c.height <= 0 || (int64_t)c.width * c.height > (int64_t)1 << 30)
    return fail(ctx, RGX_ERR_INVALID_ARG, "camera size out of range");
  if (c.width > 65535 * 8 || c.height > 65535 * 8)
    return fail(ctx, RGX_ERR_INVALID_ARG, "camera too large");
  if (!(c.fx != 0.0f) || !(c.fy != 0.0f)) return fail(ctx, RGX_ERR_INVALID_ARG, "zero focal length");
  if (!(c.t_near >= 0.0f) || !(c.t_far > c.t_near))
    return fail(ctx, RGX_ERR_INVALID_ARG, "need 0 <= t_near < t_far");
  for (int i = 0; i < 12; i++)
    if (!std::isfinite(c.cam_to_world[i])) return fail(ctx, RGX_ERR_INVALID_ARG, "non-finite pose");
  return RGX_OK;
}

static uint32_t interleave2(uint32_t x, uint32_t y) {
  uint32_t r = 0;
  for (int b = 0; b < 16; b++) r |= ((x >> b) & 1u) << (2 * b) | ((y >> b) & 1u) << (2 * b + 1);
  return r;
}

// Tile coordinates of a view in Morton order of (tx, ty), cached per shape.
static rgx_status tile_order(rgx_context *ctx, int W, int H, int tw, int th, const int32_t **out) {
  auto key = std::make_tuple(W, H, tw, th);
  auto it = ctx->tile_orders.find(key);
  if (it != ctx->tile_orders.end()) { *out = it->second; return RGX_OK; }
  const int tx = (W + tw - 1) / tw, ty = (H + th - 1) / th;
  std::vector<std::pair<uint32_t, int32_t>> v;
  v.reserve((size_t)tx * ty);
  for (int y = 0; y < ty; y++)
    for (int x = 0; x < tx; x++) v.push_back({interleave2(x, y), x | (y << 16)});
  std::sort(v.begin(), v.end());
  std::vector<int32_t> codes(v.size());
  for (size_t i = 0; i < v.size(); i++) codes[i] = v[i].second;
  int32_t *d = nullptr;
  HIP_TRY(ctx, hipMalloc(&d, codes.size() * sizeof(int32_t)));
  HIP_TRY(ctx, hipMemcpy(d, codes.data(), codes.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  ctx->tile_orders[key] = d;
  *out = d;
  return RGX_OK;
}

// Split the views into launches of at most kMaxViewsPerLaunch.
static rgx_status view_tables(rgx_context *ctx, const rgx_camera *cams, int n_views,
                              const MarchOpts &m, std::vector<ViewTable> &tabs,
                              int64_t ray0 = 0, int64_t tile0 = 0) {
  if (!cams || n_views <= 0) return fail(ctx, RGX_ERR_INVALID_ARG, "no views");
  int64_t ray = ray0, tile_base = tile0;
  for (int v0 = 0; v0 < n_views; v0 += kMaxViewsPerLaunch) {
    ViewTable t;
    memset(&t, 0, sizeof t);
    int tiles = 0;
    for (int v = v0; v < std::min(n_views, v0 + kMaxViewsPerLaunch); v++) {
      const rgx_camera &c = cams[v];
      rgx_status s = check_camera(ctx, c);
      if (s != RGX_OK) return s;
      View &V = t.v[t.n_views++];
      V.width = c.width;
      V.height = c.height;
      if (m.ray_order == 0) {
        V.tiles_x = (c.width * c.height + 63) / 64;
        V.tiles_y = 1;
        V.tile_order = nullptr;
      } else {
        V.tiles_x = (c.width + m.tile_w - 1) / m.tile_w;
        V.tiles_y = (c.height + m.tile_h - 1) / m.tile_h;
        s = tile_order(ctx, c.width, c.height, m.tile_w, m.tile_h, &V.tile_order);
        if (s != RGX_OK) return s;
      }
      {
        // every segment must advance in FP32 up to t_far: its length N_s dt
        // (at least N_s dt_min in adaptive mode) above twice the spacing of
        // floats near t_far, so that a + N_s dt > a for every a < t_far
        const double seg_min = (double)m.n_s * (m.adaptive ? m.dt_min : m.dt);
        if (seg_min < std::ldexp((double)c.t_far, -21))
          return fail(ctx, RGX_ERR_INVALID_ARG, "segment length below the FP32 resolution at t_far");
      }
      if (!m.adaptive) {
        // fixed-step sample positions come from exact integer-to-float products
        const double segs = ((double)c.t_far - (double)c.t_near) / ((double)m.dt * m.n_s);
        if (segs > (double)(1 << 22))
          return fail(ctx, RGX_ERR_INVALID_ARG, "(t_far - t_near) / (dt * n_s) exceeds 2^22");
      }
      V.tile_begin = tiles;
      if (ray > INT32_MAX - (int64_t)c.width * c.height)
        return fail(ctx, RGX_ERR_INVALID_ARG, "too many rays in one call");
      V.ray_begin = (int32_t)ray;
      tiles += V.tiles_x * V.tiles_y;
      ray += (int64_t)c.width * c.height;
      V.fx = c.fx; V.fy = c.fy; V.cx = c.cx; V.cy = c.cy;
      memcpy(V.c2w, c.cam_to_world, sizeof V.c2w);
      V.t_near = c.t_near;
      V.t_far = c.t_far;
    }
    t.n_tiles = tiles;
    if (tile_base > INT32_MAX - tiles) return fail(ctx, RGX_ERR_INVALID_ARG, "too many tiles in one call");
    t.tile0 = (int32_t)tile_base;
    tile_base += tiles;
    tabs.push_back(t);
  }
  return RGX_OK;
}

// Grows a state's record buffer to at least `need` bytes; an outgrown buffer
// is kept until rgx_fwd_destroy (a captured graph may hold its address).
static bool grow_record(rgx_fwd *f, DevBuf &b, size_t need) {
  if (b.bytes >= need) return true;
  void *p = nullptr;
  const size_t bytes = std::max(need, 2 * b.bytes);
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();   // an allocation failure only disables the record
    return false;
  }
  if (b.p) f->retired.push_back(b.p);
  b.p = p;
  b.bytes = bytes;
  return true;
}

static int64_t total_rays(const rgx_camera *cams, int32_t n_views) {
  int64_t r = 0;
  for (int v = 0; v < n_views; v++) r += (int64_t)cams[v].width * cams[v].height;
  return r;
}

// waves_per_cu: how many of the kernel's one-wave workgroups fit on a CU
static LaunchShape shape_for(rgx_context *ctx, const MarchOpts &m, int n_tiles, int waves_per_cu) {
  LaunchShape ls;
  ls.queue = ctx->queue;
  ls.error_flag = ctx->queue + 8;
  // one wave (one 64-ray tile) per workgroup
  ls.grid = m.persistent ? std::min(n_tiles, ctx->n_cu * waves_per_cu) : n_tiles;
  if (ls.grid < 1) ls.grid = 1;
  return ls;
}

extern "C" {

rgx_status rgx_render_forward(rgx_context *ctx, const rgx_bvh *bvh, const rgx_camera *cams,
                              int32_t n_views, const rgx_render_opts *opts, float *out_rgb,
                              float *out_T, int32_t *stats, rgx_fwd **state, hipStream_t stream) {
  if (!ctx || !bvh || !out_rgb || !out_T) return fail(ctx, RGX_ERR_INVALID_ARG, "null argument");
  if (bvh->ctx != ctx) return fail(ctx, RGX_ERR_STATE, "structure built on another context");
  if (state && *state && (*state)->ctx != ctx)
    return fail(ctx, RGX_ERR_STATE, "forward state of another context");
  MarchOpts m;
  rgx_status s = make_opts(ctx, bvh, opts, m);
  if (s != RGX_OK) return s;
  HIP_TRY(ctx, enter(ctx->device));
  std::vector<ViewTable> tabs;
  if ((s = view_tables(ctx, cams, n_views, m, tabs)) != RGX_OK) return s;
  const SceneDev sd = scene_of(bvh);
  FwdOut out;
  memset(&out, 0, sizeof out);
  out.rgb = out_rgb;
  out.T = out_T;
  out.stats = stats;
  int64_t tiles = 0;
  for (const ViewTable &t : tabs) tiles += t.n_tiles;
  const int64_t rays = total_rays(cams, n_views);
  rgx_fwd *f = nullptr;
  if (state) {
    f = *state ? *state : new rgx_fwd();
    f->ctx = ctx;
    f->device = ctx->device;
    f->bvh = bvh;
    f->serial = bvh->serial;
    f->n = bvh->n;
    f->cams.assign(cams, cams + n_views);
    f->opts = *opts;
    f->rays = rays;
    f->tiles = tiles;
    f->recorded = false;
    f->has_totals = false;
    // record the searches for the backward: each ray's first closest-hit
    // results, every window list of every tile and each segment step's
    // per-sample sums
    const size_t need = (size_t)rays * kReplayK * sizeof(float);
    // a shared pool: 48 KB per tile on average for the window lists, as much
    // again for the per-sample sums at N_s <= 8 (twice that at 16), at least
    // 64 MB so that a call of few tiles with long window lists still records
    // them all
    const bool samples = !opts->no_sample_record;
    const size_t per_tile = (size_t)kWrecDwordsPerTile +
                            (samples ? (size_t)kSrecDwordsPerTile * (m.n_s > 8 ? 2 : 1) : 0);
    size_t pool = std::min<size_t>(
        std::max<size_t>(2 + (size_t)tiles * per_tile, (size_t)1 << 24), 0xfffffff0u);
    // a caller's cap (the two counter dwords always fit)
    if (ctx->record_limit > 0)
      pool = std::max<size_t>(std::min<size_t>(pool, (size_t)ctx->record_limit / sizeof(uint32_t)), 2);
    if (m.ess && !m.brute_force && !opts->no_record && grow_record(f, f->replay, need) &&
        grow_record(f, f->wrec, pool * sizeof(uint32_t)) &&
        grow_record(f, f->wrec_tile, (size_t)tiles * 2 * sizeof(uint32_t))) {
      m.replay_mode = 1;
      m.replay = (float *)f->replay.p;
      m.wrec = (uint32_t *)f->wrec.p;
      m.wrec_tile = (uint32_t *)f->wrec_tile.p;
      m.wrec_cap = (uint32_t)pool;
      m.sample_rec = samples ? 1 : 0;
      // the pool's 64-bit allocation counter (dwords 0-1) starts past itself
      // (fill kernels, not memset nodes, so the call can be captured)
      hipError_t e = launch_fill(f->wrec.p, 1, 2u, stream);
      if (e == hipSuccess) e = launch_fill((uint32_t *)f->wrec.p + 1, 1, 0u, stream);
      if (e != hipSuccess) {
        if (!*state) rgx_fwd_destroy(f);
        return hip_fail(ctx, e, "record reset");
      }
      f->recorded = true;
    }
    if (stats && !grow_record(f, f->totals, RGX_NTOT * sizeof(int64_t))) {
      if (!*state) rgx_fwd_destroy(f);
      return fail(ctx, RGX_ERR_OUT_OF_MEMORY, "statistics totals");
    }
    *state = f;
  }
  for (const ViewTable &t : tabs) {
    if (t.n_tiles == 0) continue;
    HIP_TRY(ctx, timed(ctx, RGX_KERN_FORWARD, stream,
                       [&] { return launch_forward(sd, t, m, out, shape_for(ctx, m, t.n_tiles, fwd_waves_per_cu(m)), stream); }));
  }
  if (f && stats) {
    HIP_TRY(ctx, launch_stat_totals(stats, rays, sd, f->recorded ? (const uint32_t *)f->wrec_tile.p : nullptr,
                                    tiles, (int64_t *)f->totals.p, stream));
    f->has_totals = true;
  }
  return RGX_OK;
}

rgx_status rgx_render_backward(rgx_context *ctx, const rgx_bvh *bvh, const rgx_fwd *f,
                               const float *out_rgb, const float *out_T, const float *grad_rgb,
                               const float *grad_T, const rgx_grads *grads, hipStream_t stream) {
  if (!ctx || !bvh || !f || !out_rgb || !out_T || !grad_rgb || !grads)
    return fail(ctx, RGX_ERR_INVALID_ARG, "null argument");
  if (!grads->means || !grads->log_scales || !grads->quats || !grads->density || !grads->sh)
    return fail(ctx, RGX_ERR_INVALID_ARG, "null gradient buffer");
  if (f->ctx != ctx || bvh->ctx != ctx) return fail(ctx, RGX_ERR_STATE, "state of another context");
  if (f->bvh != bvh || f->serial != bvh->serial)
    return fail(ctx, RGX_ERR_STATE, "the structure was rebuilt or replaced since the forward");
  if (grads->n != bvh->n) return fail(ctx, RGX_ERR_INVALID_ARG, "gradient buffers do not match the structure's n");
  if (bvh->n_sg > 0 && !grads->sg) return fail(ctx, RGX_ERR_INVALID_ARG, "the structure has lobes: grads->sg needed");
  const rgx_camera *cams = f->cams.data();
  const int32_t n_views = (int32_t)f->cams.size();
  MarchOpts m;
  rgx_status s = make_opts(ctx, bvh, &f->opts, m);
  if (s != RGX_OK) return s;
  HIP_TRY(ctx, enter(ctx->device));
  std::vector<ViewTable> tabs;
  if ((s = view_tables(ctx, cams, n_views, m, tabs)) != RGX_OK) return s;
  const SceneDev sd = scene_of(bvh);
  // the accumulators are zero: cleared by the build and by every finalisation
  ctx->replayed = 0;
  if (f->recorded) {
    m.replay_mode = 2;
    m.replay = (float *)f->replay.p;
    m.wrec = (uint32_t *)f->wrec.p;
    m.wrec_tile = (uint32_t *)f->wrec_tile.p;
    m.wrec_cap = (uint32_t)std::min<size_t>(f->wrec.bytes / sizeof(uint32_t), 0xfffffff0u);
    m.sample_rec = f->opts.no_sample_record ? 0 : 1;
    ctx->replayed = 1;
  }
  BwdIn in;
  in.rgb = out_rgb;
  in.T = out_T;
  in.grad_rgb = grad_rgb;
  in.grad_T = grad_T;
  in.acc = (float *)bvh->acc.p;
  in.sgacc = bvh->n_sg > 0 ? (float *)bvh->sgacc.p : nullptr;
  if (!grads->densify) {
    for (const ViewTable &t : tabs) {
      if (t.n_tiles == 0) continue;
      HIP_TRY(ctx, timed(ctx, RGX_KERN_BACKWARD, stream,
                         [&] { return launch_backward(sd, t, m, in, shape_for(ctx, m, t.n_tiles, bwd_waves_per_cu(m)), stream); }));
    }
  } else {
    // one view at a time: each view's mean gradient is the change of the
    // accumulated mean slots, turned into the densification statistic
    if (!grads->densify_views) return fail(ctx, RGX_ERR_INVALID_ARG, "densify needs densify_views");
    rgx_bvh *mb = const_cast<rgx_bvh *>(bvh);
    HIP_TRY(ctx, ensure(mb->zsum, (size_t)bvh->n * 3 * sizeof(float)));
    HIP_TRY(ctx, launch_fill(mb->zsum.p, bvh->n * 3, 0u, stream));
    int64_t ray0 = 0, tile0 = 0;
    for (int v = 0; v < n_views; v++) {
      std::vector<ViewTable> one;
      if ((s = view_tables(ctx, cams + v, 1, m, one, ray0, tile0)) != RGX_OK) return s;
      ray0 += (int64_t)cams[v].width * cams[v].height;
      tile0 += one[0].n_tiles;
      for (const ViewTable &t : one) {
        if (t.n_tiles == 0) continue;
        HIP_TRY(ctx, timed(ctx, RGX_KERN_BACKWARD, stream,
                           [&] { return launch_backward(sd, t, m, in, shape_for(ctx, m, t.n_tiles, bwd_waves_per_cu(m)), stream); }));
      }
      const float *c2w = cams[v].cam_to_world;
      HIP_TRY(ctx, launch_densify(sd, (float *)bvh->acc.p, (float *)mb->zsum.p, c2w[3], c2w[7],
                                  c2w[11], cams[v].fx, grads->densify, grads->densify_views, stream));
    }
    HIP_TRY(ctx, launch_densify_restore(sd, (float *)bvh->acc.p, (const float *)mb->zsum.p, stream));
  }
  HIP_TRY(ctx, timed(ctx, RGX_KERN_FINALIZE, stream, [&] {
    return launch_finalize_grads(sd, bvh->sh_k, (float *)bvh->acc.p, grads->means, grads->log_scales,
                                 grads->quats, grads->density, grads->sh, grads->accumulate, stream);
  }));
  if (bvh->n_sg > 0)
    HIP_TRY(ctx, launch_finalize_sg(sd, (float *)bvh->sgacc.p, grads->sg, grads->accumulate, stream));
  return RGX_OK;
}

void rgx_fwd_destroy(rgx_fwd *f) {
  if (!f) return;
  (void)hipSetDevice(f->device);
  release(f->replay);
  release(f->wrec);
  release(f->wrec_tile);
  release(f->totals);
  for (void *p : f->retired) (void)hipFree(p);
  delete f;
}

rgx_status rgx_sync_stats(rgx_context *ctx, const rgx_fwd *f, int64_t *out, hipStream_t stream) {
  if (!ctx || !f || !out) return fail(ctx, RGX_ERR_INVALID_ARG, "null argument");
  if (f->ctx != ctx) return fail(ctx, RGX_ERR_STATE, "state of another context");
  if (!f->has_totals) return fail(ctx, RGX_ERR_STATE, "the forward was not given a stats buffer");
  HIP_TRY(ctx, enter(ctx->device));
  HIP_TRY(ctx, hipStreamSynchronize(stream));
  HIP_TRY(ctx, hipMemcpy(out, f->totals.p, RGX_NTOT * sizeof(int64_t), hipMemcpyDeviceToHost));
  return RGX_OK;
}

rgx_status rgx_dump_hits(rgx_context *ctx, const rgx_bvh *bvh, const rgx_camera *cam,
                         const rgx_render_opts *opts, const int32_t *pix, int32_t n_rays,
                         int32_t cap, float *seg_a, int32_t *ids, int32_t *count,
                         hipStream_t stream) {
  if (!ctx || !bvh || !cam || !pix || !seg_a || !ids || !count || n_rays <= 0 || cap <= 0)
    return fail(ctx, RGX_ERR_INVALID_ARG, "bad argument");
  MarchOpts m;
  rgx_status s = make_opts(ctx, bvh, opts, m);
  if (s != RGX_OK) return s;
  m.persistent = 0;
  HIP_TRY(ctx, enter(ctx->device));
  if ((s = check_camera(ctx, *cam)) != RGX_OK) return s;
  ViewTable t;
  memset(&t, 0, sizeof t);
  t.n_views = 1;
  View &V = t.v[0];
  V.width = cam->width; V.height = cam->height;
  V.fx = cam->fx; V.fy = cam->fy; V.cx = cam->cx; V.cy = cam->cy;
  memcpy(V.c2w, cam->cam_to_world, sizeof V.c2w);
  V.t_near = cam->t_near; V.t_far = cam->t_far;
  t.n_tiles = (n_rays + 63) / 64;
  FwdOut out;
  memset(&out, 0, sizeof out);
  out.dump_pix = pix;
  out.dump_n = n_rays;
  out.dump_cap = cap;
  out.dump_a = seg_a;
  out.dump_ids = ids;
  out.dump_count = count;
  HIP_TRY(ctx, launch_forward(scene_of(bvh), t, m, out, shape_for(ctx, m, t.n_tiles, fwd_waves_per_cu(m)), stream));
  return RGX_OK;
}

rgx_status rgx_false_positives(rgx_context *ctx, const rgx_bvh *bvh, const rgx_camera *cam,
                               const int32_t *pix, int32_t n_rays, const float *t_end,
                               int32_t *count, hipStream_t stream) {
  if (!ctx || !bvh || !cam || !pix || !t_end || !count || n_rays <= 0)
    return fail(ctx, RGX_ERR_INVALID_ARG, "bad argument");
  if (bvh->ctx != ctx) return fail(ctx, RGX_ERR_STATE, "structure built on another context");
  rgx_status s = check_camera(ctx, *cam);
  if (s != RGX_OK) return s;
  HIP_TRY(ctx, enter(ctx->device));
  View V;
  memset(&V, 0, sizeof V);
  V.width = cam->width; V.height = cam->height;
  V.fx = cam->fx; V.fy = cam->fy; V.cx = cam->cx; V.cy = cam->cy;
  memcpy(V.c2w, cam->cam_to_world, sizeof V.c2w);
  V.t_near = cam->t_near; V.t_far = cam->t_far;
  HIP_TRY(ctx, launch_false_positives(scene_of(bvh), V, pix, n_rays, t_end, count, ctx->queue + 8, stream));
  return RGX_OK;
}

rgx_status rgx_bvh_debug(rgx_context *ctx, const rgx_bvh *b, uint64_t *keys, int32_t *perm,
                         float *aabb, float *nodes, float *nodes4, int64_t *n_active,
                         hipStream_t stream) {
  if (!ctx || !b) return fail(ctx, RGX_ERR_INVALID_ARG, "null argument");
  HIP_TRY(ctx, enter(ctx->device));
  HIP_TRY(ctx, hipStreamSynchronize(stream));
  const size_t n = (size_t)b->n;
  if (keys)
    HIP_TRY(ctx, hipMemcpy(keys, b->sorted_sel ? b->keys1.p : b->keys0.p, n * 8, hipMemcpyDeviceToHost));
  if (perm)
    HIP_TRY(ctx, hipMemcpy(perm, b->sorted_sel ? b->vals1.p : b->vals0.p, n * 4, hipMemcpyDeviceToHost));
  if (aabb) HIP_TRY(ctx, hipMemcpy(aabb, b->aabb.p, n * 24, hipMemcpyDeviceToHost));
  if (nodes)
    HIP_TRY(ctx, hipMemcpy(nodes, b->nodes.p, std::max<size_t>(n - 1, 1) * 64, hipMemcpyDeviceToHost));
  if (nodes4)
    HIP_TRY(ctx, hipMemcpy(nodes4, b->nodes4.p, std::max<size_t>(n - 1, 1) * kNode4Floats * 4,
                           hipMemcpyDeviceToHost));
  if (n_active) {
    int32_t c = 0;
    HIP_TRY(ctx, hipMemcpy(&c, b->counters.p, 4, hipMemcpyDeviceToHost));
    *n_active = c;
  }
  return RGX_OK;
}

rgx_status rgx_set_record_limit(rgx_context *ctx, int64_t max_bytes) {
  if (!ctx) return RGX_ERR_INVALID_ARG;
  if (max_bytes < 0) return fail(ctx, RGX_ERR_INVALID_ARG, "negative record limit");
  ctx->record_limit = max_bytes;
  return RGX_OK;
}

rgx_status rgx_set_kernel_timing(rgx_context *ctx, int32_t enable) {
  if (!ctx) return RGX_ERR_INVALID_ARG;
  ctx->timing = enable != 0;
  ctx->ev_used = 0;
  return RGX_OK;
}

rgx_status rgx_kernel_times(rgx_context *ctx, double *ms, int64_t *launches, int32_t reset) {
  if (!ctx || !ms || !launches) return fail(ctx, RGX_ERR_INVALID_ARG, "null argument");
  for (int k = 0; k < RGX_NKERN; k++) { ms[k] = 0.0; launches[k] = 0; }
  HIP_TRY(ctx, enter(ctx->device));
  for (size_t i = 0; i < ctx->ev_used; i += 2) {
    HIP_TRY(ctx, hipEventSynchronize(ctx->ev[i + 1]));
    float t = 0.0f;
    HIP_TRY(ctx, hipEventElapsedTime(&t, ctx->ev[i], ctx->ev[i + 1]));
    const int k = ctx->ev_kind[i / 2];
    ms[k] += t;
    launches[k] += 1;
  }
  if (reset) ctx->ev_used = 0;
  return RGX_OK;
}

rgx_status rgx_isotropic_loss(rgx_context *ctx, int64_t n, const float *log_scales, float r0,
                              float *loss, float *grad, int32_t accumulate, hipStream_t stream) {
  if (!ctx || !log_scales || !loss || !grad) return fail(ctx, RGX_ERR_INVALID_ARG, "null argument");
  if (n <= 0 || n > RGX_MAX_GAUSSIANS) return fail(ctx, RGX_ERR_INVALID_ARG, "n out of range");
  if (!(r0 > 0.0f) || !std::isfinite(r0)) return fail(ctx, RGX_ERR_INVALID_ARG, "r0 must be > 0");
  HIP_TRY(ctx, enter(ctx->device));
  const int64_t nb = iso_blocks(n);
  if (nb > ctx->partial_cap) {
    if (ctx->partial) (void)hipFree(ctx->partial);
    ctx->partial = nullptr;
    ctx->partial_cap = 0;
    HIP_TRY(ctx, hipMalloc((void **)&ctx->partial, (size_t)nb * sizeof(double)));
    ctx->partial_cap = nb;
  }
  HIP_TRY(ctx, launch_isotropic_loss(n, log_scales, r0, loss, grad, accumulate, ctx->partial, stream));
  return RGX_OK;
}

rgx_status rgx_isotropic_loss_noalloc(rgx_context *ctx, int64_t n, const float *log_scales,
                                      float r0, float *loss, float *grad, int32_t accumulate,
                                      hipStream_t stream) {
  if (!ctx || !log_scales || !loss || !grad) return fail(ctx, RGX_ERR_INVALID_ARG, "null argument");
  if (n <= 0 || n > RGX_MAX_GAUSSIANS) return fail(ctx, RGX_ERR_INVALID_ARG, "n out of range");
  if (iso_blocks(n) > iso_scratch_capacity())
    return fail(ctx, RGX_ERR_INVALID_ARG, "n exceeds the fixed workspace of the allocation-free loss");
  if (!(r0 > 0.0f) || !std::isfinite(r0)) return fail(ctx, RGX_ERR_INVALID_ARG, "r0 must be > 0");
  if (!ctx->iso_scratch) return fail(ctx, RGX_ERR_STATE, "fixed workspace address not resolved");
  HIP_TRY(ctx, enter(ctx->device));
  HIP_TRY(ctx, launch_isotropic_loss(n, log_scales, r0, loss, grad, accumulate, ctx->iso_scratch, stream));
  return RGX_OK;
}

rgx_status rgx_adam_step(rgx_context *ctx, const rgx_adam_group *groups, int32_t n_groups,
                         int32_t *step, float beta1, float beta2, float eps, hipStream_t stream) {
  if (!ctx || !groups || !step || n_groups < 1) return fail(ctx, RGX_ERR_INVALID_ARG, "bad argument");
  if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return fail(ctx, RGX_ERR_INVALID_ARG, "need 0 <= beta < 1 and eps > 0");
  for (int32_t k = 0; k < n_groups; k++) {
    const rgx_adam_group &g = groups[k];
    if (g.n < 0 || (g.n > 0 && (!g.param || !g.grad || !g.m || !g.v)) || !std::isfinite(g.lr))
      return fail(ctx, RGX_ERR_INVALID_ARG, "bad Adam group");
  }
  HIP_TRY(ctx, enter(ctx->device));
  HIP_TRY(ctx, launch_adam_tick(step, stream));
  for (int32_t k = 0; k < n_groups; k++) {
    const rgx_adam_group &g = groups[k];
    HIP_TRY(ctx, launch_adam(g.n, g.param, g.grad, g.m, g.v, g.lr, beta1, beta2, eps, step, stream));
  }
  return RGX_OK;
}

rgx_status rgx_error_flags(rgx_context *ctx, int32_t *flags, hipStream_t stream) {
  if (!ctx || !flags) return fail(ctx, RGX_ERR_INVALID_ARG, "null argument");
  HIP_TRY(ctx, enter(ctx->device));
  HIP_TRY(ctx, hipStreamSynchronize(stream));
  HIP_TRY(ctx, hipMemcpy(flags, ctx->queue + 8, 4, hipMemcpyDeviceToHost));
  return RGX_OK;
}

}  // extern "C"

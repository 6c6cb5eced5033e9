// Shared device-side definitions of the gfx950 ray-marching library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rgx {

constexpr int kWave = 64;
constexpr int kBlock = 256;               // 4 waves, each owning its own 64-ray tile
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kMaxViewsPerLaunch = 24;    // view table travels as a kernel argument
constexpr int kGeomFloats = 16;           // packed geometry record (64 B)
constexpr int kAccFloats = 64;            // per-Gaussian gradient accumulator (256 B)
constexpr int kColFloats = 48;            // colour record: 3 x 16 SH coefficients, zero past the degree
// 4-wide node record: 4 child boxes (lo xyz, hi xyz), 4 child links (>= 0
// 4-wide node, < 0 leaf ~j, kNoChild none), 4 leaf ranges (first, last).
constexpr int kNode4Floats = 36;
constexpr int kAuxFloats = 8;             // s.xyz, unit quaternion (w,x,y,z), |q|
// Spherical-Gaussian colour lobes (the 9 SH + 7 SG appearance model): up to
// kMaxSg lobes per Gaussian, kSgLobeFloats per lobe in the packed record:
// amplitude rgb, sharpness lambda, unit axis xyz, |xi| (0: lobe absent).
constexpr int kMaxSg = 7;
constexpr int kSgLobeFloats = 8;
constexpr int kSgFloats = kMaxSg * kSgLobeFloats;   // 56
constexpr int kSgUserFloats = 7;          // user lobe: amplitude rgb, axis xyz, sharpness
constexpr int kSgAccFloats = 64;          // per Gaussian: 8 slots per lobe (da rgb, dlambda, h xyz, pad)
constexpr int32_t kNoChild = INT32_MIN;

// Packed geometry record, Z order: [mu.xyz, k^2, M (3x3 row-major), sigma~, log2 sigma~, pad]
// with M = S^-1 R^T so that q = |M (x - mu)|^2.
// G_RAD: radius of a sphere around the mean holding the whole ellipsoid
enum GeomSlot { G_MU = 0, G_K2 = 3, G_M = 4, G_SIG = 13, G_L2SIG = 14, G_RAD = 15 };

// per-ray statistics slots (same order as the public RGX_STAT_* enum)
enum { ST_Q = 0, ST_P, ST_SAMPLES, ST_SEGMENTS, ST_CLOSEST, ST_BOX_ONLY, ST_NODES, ST_LEAVES,
       ST_WINDOWS, ST_CHUNKED, ST_CAND, ST_CAND_HIT, ST_KCYC_COLLECT, ST_KCYC_CLOSEST,
       ST_KCYC_TILE, ST_T_END };
constexpr int kNStatUsed = 16;
constexpr int kNStat = 16;

struct View {
  const int32_t *tile_order;  // tile coordinates (tx | ty << 16) in launch order
  int32_t width, height, tiles_x, tiles_y;
  int32_t tile_begin;     // first global tile index of the view
  int32_t ray_begin;      // first output ray of the view
  float fx, fy, cx, cy;
  float c2w[12];
  float t_near, t_far;
};

struct ViewTable {
  int32_t n_views;
  int32_t n_tiles;        // total tiles over the views of this launch
  int32_t tile0;          // index of this launch's first tile among all tiles of the call
  View v[kMaxViewsPerLaunch];
};

struct MarchOpts {
  int32_t adaptive;
  float dt, dt_min, dt_max, inv_beta;
  int32_t n_s;
  float t_eps;
  int32_t ess;
  int32_t brute_force;
  int32_t ray_order;
  int32_t tile_w, tile_h, tile_w_log2;
  int32_t persistent;
  int32_t window_segments;
  float bg[3];
  int32_t sh_k;           // SH coefficients per channel
  int32_t col_stride;     // floats per packed colour record
  // closest-hit replay: the forward records each ray's first kReplayK
  // closest-hit results, a backward of the same rays replays them
  int32_t replay_mode;    // 0 off, 1 record, 2 replay
  float *replay;          // [rays of the call][kReplayK]
  uint32_t *wrec;         // window-list record pool: [0,2) 64-bit allocation counter, records after
  uint32_t *wrec_tile;    // per tile of the call: (complete, first chunk offset)
  uint32_t wrec_cap;      // pool size in dwords
  int32_t sample_rec;     // the record also holds each segment step's per-sample sums
};
constexpr int kReplayK = 4;
// Window-list record: every collection of a tile appends one chunk to a
// shared pool (offsets in dwords): a header (count returned, paused, z0, z1,
// zp, list size, offset of the tile's next chunk) and that many (id, t_in,
// t_out) entries in Z order.  A tile whose chunks do not all fit is marked
// incomplete and is not replayed.
constexpr int kWrecHeader = 7;
constexpr uint32_t kWrecNone = 0xffffffffu;
// Sample record: after every segment step of a tile the forward appends
// [next, hit-lane mask (2 dwords), empty-lane mask (2 dwords)], then for the
// lanes whose segment hit some Gaussian the per-sample sums sigma_k and the
// colour sum W_k (4 N_S floats per lane, stored as [k][component][lane rank]),
// then for the lanes whose segment was empty the restart distance it found.
constexpr int kSrecHeader = 5;
// pool size per tile of the call (average): window lists, and with them the
// sample records
constexpr int kWrecDwordsPerTile = 12288;
constexpr int kSrecDwordsPerTile = 12288;

// Scalar (constant address space) views of read-only scene data: a
// wave-uniform address loads once into SGPRs for the whole wave.
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) vf4 *cfloat4p;
typedef const __attribute__((address_space(4))) float *cfloatp;
typedef const __attribute__((address_space(4))) int32_t *cintp;

__device__ __forceinline__ cfloat4p as_const4(const float *p) {
  return (cfloat4p)(const __attribute__((address_space(4))) void *)(uintptr_t)p;
}
__device__ __forceinline__ cfloatp as_constf(const float *p) {
  return (cfloatp)(const __attribute__((address_space(4))) void *)(uintptr_t)p;
}

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uniform_float(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Real SH basis (Condon-Shortley phase, index l^2+l+m) at a unit direction,
// as polynomials in (x, y, z) for degrees 0..3; entries m >= k are zero.
__device__ __forceinline__ void sh_basis(int k, float x, float y, float z, float *Y) {
#pragma unroll
  for (int m = 1; m < 16; m++) Y[m] = 0.0f;
  Y[0] = 0.28209479177387814f;
  if (k <= 1) return;
  Y[1] = -0.48860251190291992f * y;
  Y[2] = 0.48860251190291992f * z;
  Y[3] = -0.48860251190291992f * x;
  if (k <= 4) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = 1.0925484305920792f * x * y;
  Y[5] = -1.0925484305920792f * y * z;
  Y[6] = 0.31539156525252005f * (2.0f * zz - xx - yy);
  Y[7] = -1.0925484305920792f * x * z;
  Y[8] = 0.54627421529603959f * (xx - yy);
  if (k <= 9) return;
  Y[9] = -0.59004358992664352f * y * (3.0f * xx - yy);
  Y[10] = 2.8906114426405538f * x * y * z;
  Y[11] = -0.45704579946446572f * y * (4.0f * zz - xx - yy);
  Y[12] = 0.37317633259011540f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
  Y[13] = -0.45704579946446572f * x * (4.0f * zz - xx - yy);
  Y[14] = 1.4453057213202769f * z * (xx - yy);
  Y[15] = -0.59004358992664352f * x * (xx - 3.0f * yy);
}

constexpr float kLog2e = 1.4426950408889634f;

// exp(-x) through the hardware base-2 exponential.
__device__ __forceinline__ float exp_neg(float x) { return __builtin_amdgcn_exp2f(-x * kLog2e); }

// 1 - exp(-x) for x >= 0 without cancellation at small x.
__device__ __forceinline__ float one_minus_exp_neg(float x) {
  const float e = exp_neg(x);
  const float series = x * (1.0f - x * (0.5f - x * (1.0f / 6.0f)));
  return x < 1e-3f ? series : 1.0f - e;
}

}  // namespace rgx

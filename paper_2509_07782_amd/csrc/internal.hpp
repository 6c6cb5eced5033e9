// Host-side launch interfaces between the C ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace rgx {

struct BuildArgs {
  int64_t n;
  const float *means, *log_scales, *quats, *density, *sh;
  const float *sg;           // [n, n_sg, 7] user lobes (n_sg > 0)
  int n_sg;
  float *sg_user, *sgrec;    // packed lobes, user order / Z order [n, kSgFloats]
  int sh_k, col_stride, morton_bits;
  float sigma_eps;
  // scratch (user order)
  float *geom_user, *aabb_user, *aux_user;
  uint8_t *active;
  uint32_t *bounds;          // 6 ordered floats
  int32_t *counters;         // [0] active count
  uint64_t *keys[2];
  uint32_t *vals[2];
  uint32_t *sort_hist;
  int *sorted_sel;           // (host) which ping-pong buffer holds the result
  // outputs (Z order)
  float *geom, *aabb, *col, *aux, *nodes;
  float *nodes4;             // 4-wide nodes, one per binary internal node, same index
  float *seg;                // segment tree of leaf boxes, 2P boxes
};
hipError_t launch_build(const BuildArgs &a, hipStream_t st);
int64_t iso_blocks(int64_t n);
// Largest n (must equal RGX_MAX_GAUSSIANS of the public header).
constexpr int64_t RGX_MAX_GAUSSIANS_INTERNAL = int64_t(1) << 23;
// Per-device fixed partial-sum workspace of rgx_isotropic_loss_noalloc:
// capacity in doubles, and its device address on the current device.
int64_t iso_scratch_capacity();
hipError_t iso_scratch_resolve(double **ptr);
hipError_t launch_isotropic_loss(int64_t n, const float *log_scales, float r0, float *loss,
                                 float *grad, int accumulate, double *partial, hipStream_t st);

struct SceneDev {
  const float *geom;          // [n,16]
  const float *col;           // [n,col_stride]
  const float *nodes;         // [max(n-1,1),16]
  const float *nodes4;        // [max(n-1,1),36] 4-wide nodes, one per binary internal node
  const float *aabb;          // [n,6]
  const int32_t *counters;    // [0] = active count
  const uint32_t *perm;       // Z index -> user index
  const float *aux;           // [n,8] s.xyz, unit quaternion wxyz, |q| (Z order)
  const float *sg;            // [n, kSgFloats] packed lobes (Z order), nullptr without lobes
  int n_sg;
  int64_t n;
};

struct FwdOut {
  float *rgb, *T;
  int32_t *stats;            // nullable
  // hit dump (debug)
  const int32_t *dump_pix;
  int32_t dump_n, dump_cap;
  float *dump_a;
  int32_t *dump_ids, *dump_count;
};

struct BwdIn {
  const float *rgb, *T, *grad_rgb, *grad_T;
  float *acc;                // [n, 64] packed-order gradient accumulators
  float *sgacc;              // [n, kSgAccFloats] lobe accumulators (with lobes)
};

struct LaunchShape {
  int grid;
  int32_t *queue;            // persistent tile queues (8 counters), zeroed by the launch
  int32_t *error_flag;
};

// Resident one-wave workgroups per CU of the march kernels (their launch
// bounds and LDS use), used to size persistent grids.
inline int fwd_waves_per_cu(const MarchOpts &m) { return m.n_s <= 8 ? 12 : 8; }
inline int bwd_waves_per_cu(const MarchOpts &) { return 8; }
hipError_t launch_forward(const SceneDev &s, const ViewTable &vt, const MarchOpts &op,
                          const FwdOut &out, const LaunchShape &ls, hipStream_t st);
hipError_t launch_backward(const SceneDev &s, const ViewTable &vt, const MarchOpts &op,
                           const BwdIn &in, const LaunchShape &ls, hipStream_t st);
hipError_t launch_finalize_grads(const SceneDev &s, int sh_k, float *acc, float *g_means,
                                 float *g_log_scales, float *g_quats, float *g_density,
                                 float *g_sh, int accumulate, hipStream_t st);
hipError_t launch_finalize_sg(const SceneDev &s, float *sgacc, float *g_sg, int accumulate,
                              hipStream_t st);
hipError_t launch_densify(const SceneDev &s, float *acc, float *zsum, float ox, float oy,
                          float oz, float focal, float *densify, int32_t *views, hipStream_t st);
hipError_t launch_densify_restore(const SceneDev &s, float *acc, const float *zsum, hipStream_t st);
// Totals of a forward's per-ray statistics [rays, kNStat] into int64
// totals[RGX_NTOT]; wrec_tile (nullable) gives the record's per-tile status.
hipError_t launch_stat_totals(const int32_t *stats, int64_t rays, const SceneDev &s,
                              const uint32_t *wrec_tile, int64_t tiles, int64_t *totals,
                              hipStream_t st);
// Whole-ray AABB false positives of listed pixels of one view.
hipError_t launch_false_positives(const SceneDev &s, const View &v, const int32_t *pix, int32_t n_rays,
                                  const float *t_end, int32_t *count, int32_t *error_flag,
                                  hipStream_t st);
hipError_t launch_fill(void *p, int64_t n_words, uint32_t value, hipStream_t st);
hipError_t launch_adam_tick(int32_t *step, hipStream_t st);
hipError_t launch_adam(int64_t n, float *p, const float *g, float *m, float *v, float lr, float b1,
                       float b2, float eps, const int32_t *step, hipStream_t st);
hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t st);

}  // namespace rgx

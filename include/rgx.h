/*
 * rgx.h -- C ABI of the MI355X (gfx950) library for differentiable volume ray
 * marching through truncated anisotropic Gaussians found via a BVH
 * (RayGaussX, arXiv 2509.07782).
 *
 * The method: a scene of N Gaussians defines a density field
 *   sigma(x) = sum_l sigma~_l exp(-q_l(x)/2) [q_l(x) <= k_l^2],
 *   q_l(x) = (x-mu_l)^T Sigma_l^-1 (x-mu_l), Sigma_l = R_l S_l S_l^T R_l^T,
 *   k_l^2 = 2 ln(sigma~_l / sigma_eps)                    (Sec. 3.1 Eq. 1; Supp. B)
 * and a radiance field equal to the density-weighted mean of per-Gaussian
 * spherical-harmonic colours c_l(d) at the ray direction (Eq. 1).  A pixel is
 * the discrete volume-rendering sum of Eq. 3 evaluated segment by segment as in
 * Algorithm 1 (Sec. 3.2): N_s midpoint samples per segment, empty-space
 * skipping through closest-hit queries (Eq. 4), optional adaptive segment size
 * (Eq. 5) and early termination when the transmittance drops to T_eps.
 *
 * Conventions shared by every call
 *  - Pointers are DEVICE pointers unless marked (host).  The caller owns every
 *    buffer it passes; the library keeps no pointer to a caller buffer after a
 *    call returns.
 *  - Every call is asynchronous and ordered on the given hipStream_t (NULL is
 *    the default stream).  No call synchronises the host except where stated.
 *  - Parameter arrays are float32, contiguous, row-major, in the caller's
 *    ("user") Gaussian order.  Quaternions are (w,x,y,z) of any non-zero norm;
 *    scales are given as log-scales l (s = exp(l)); density is the raw
 *    sigma~ (no activation); sh is [n, K, 3] with K = (deg+1)^2, real SH basis
 *    with the Condon-Shortley phase, index l^2+l+m, evaluated at the unit ray
 *    direction, colour used as is (no offset or clamp).
 *  - Rays: pinhole through the pixel centre (u+1/2, v+1/2), pixel (0,0) top
 *    left, camera axes x right / y down / z forward, unit direction so that t
 *    is metric distance from the camera centre.  Output pixels of view v are
 *    row-major and views are concatenated in order.
 *  - Errors: host-detectable errors return a negative rgx_status before
 *    anything is enqueued.  Data-dependent cases are not errors: a Gaussian
 *    with sigma~ <= sigma_eps, a zero quaternion or a non-finite parameter is
 *    inactive (never hit, zero gradient).  HIP failures return RGX_ERR_HIP with
 *    the HIP message in rgx_last_error(); an error left pending by the
 *    caller's own earlier HIP calls is cleared on entry to a call that
 *    launches work, so it is never reported as the library's.
 */
#ifndef RGX_H
#define RGX_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RGX_OK = 0,
  RGX_ERR_INVALID_ARG = -1,
  RGX_ERR_OUT_OF_MEMORY = -2,
  RGX_ERR_HIP = -3,
  RGX_ERR_UNSUPPORTED = -4,
  RGX_ERR_STATE = -5
} rgx_status;

/* Library context: owns the device workspace and the per-device launch
   parameters.  One context per stream/thread at a time. */
typedef struct rgx_context rgx_context;

/* Acceleration structure built from one set of Gaussian parameters: the
   Z-ordered (Morton-sorted, Sec. 3.3) copy of the per-Gaussian geometry and
   colour records, the permutation to user order and the LBVH over the
   ellipsoids' minimal AABBs (Supp. B).  Rebuilding reuses its memory. */
typedef struct rgx_bvh rgx_bvh;

/* Forward state kept for the backward (Alg. 1 run forwards, then its adjoint):
   which structure build, cameras and options the forward rendered, and what
   its searches found -- each ray's first closest-hit results (Eq. 4) and every
   window list its tiles collected -- so that the backward replays them instead
   of searching again.  Owned by the caller (rgx_fwd_destroy); it holds no
   pointer to a caller buffer. */
typedef struct rgx_fwd rgx_fwd;

typedef struct {
  int64_t n;                 /* number of Gaussians, >= 1 */
  int32_t sh_degree;         /* 0..3 */
  const float *means;        /* [n,3] mu */
  const float *log_scales;   /* [n,3] l */
  const float *quats;        /* [n,4] (w,x,y,z) */
  const float *density;      /* [n]   sigma~ */
  const float *sh;           /* [n,K,3] */
  /* Optional spherical-Gaussian colour lobes (the 9 SH + 7 SG appearance
     model of the supplement's comparison with 3D-GS): the colour at unit
     direction d becomes c(d) = sum_m f_m Y_m(d) + sum_j a_j
     exp(lambda_j (xi_j.d / |xi_j| - 1)).  n_sg = 0 (sg ignored) or 1..7;
     sg [n, n_sg, 7] per lobe (a_r, a_g, a_b, xi_x, xi_y, xi_z, lambda), the
     axis of any non-zero norm (a zero axis makes the lobe absent).  Lobes
     need rgx_render_opts.n_s = 8. */
  int32_t n_sg;
  const float *sg;
} rgx_gaussians;

typedef struct {
  float sigma_eps;           /* density threshold of the truncation ellipsoid, > 0 (default 0.01) */
  int32_t morton_bits;       /* bits per axis of the Z-order key, 1..21 (default 21) */
} rgx_build_opts;

typedef struct {             /* (host) pinhole camera */
  int32_t width, height;     /* > 0 */
  float fx, fy, cx, cy;      /* intrinsics in pixels */
  float cam_to_world[12];    /* 3x4 row-major [R | centre]; R columns = camera x, y, z in world */
  float t_near, t_far;       /* integration bounds along the ray, 0 <= t_near < t_far */
} rgx_camera;

typedef struct {
  int32_t adaptive;          /* 0: fixed step dt; 1: Eq. 5 step from dt_min, dt_max, beta */
  float dt, dt_min, dt_max, beta;
  int32_t n_s;               /* samples per segment N_s: 1, 2, 4, 8 or 16 */
  float t_eps;               /* transmittance threshold T_eps >= 0, tested at segment starts */
  int32_t ess;               /* empty-space skipping: 0 off; 1 restart snapped to the segment
                                grid (fixed step; image identical to 0); 2 restart at the
                                closest hit itself (the only form used in adaptive mode) */
  int32_t brute_force;       /* 1: test every Gaussian instead of the BVH (hit-set reference) */
  int32_t ray_order;         /* 0: scanline rows of 64 rays; 1: tiles in Morton order */
  int32_t tile_w, tile_h;    /* tile shape for ray_order 1, tile_w*tile_h = 64 (0: 8x8) */
  int32_t persistent;        /* 1: persistent launch popping tiles from a device queue */
  int32_t window_segments;   /* initial depth-window length, in longest segments (0: 1);
                                tuning only, never changes results */
  float bg[3];               /* background colour added with the final transmittance */
  int32_t no_record;         /* 1: a forward given a state keeps only its cameras and options,
                                not its searches (the backward then searches again, with the
                                same results); never changes results */
  int32_t no_sample_record;  /* 1: a forward given a state records its searches but not the
                                per-sample sums (128 B per ray segment at N_s = 8): the
                                backward then evaluates every hit Gaussian again for them,
                                which halves the state's pool and costs backward time; the
                                same results up to the rounding of the colour sums */
} rgx_render_opts;

typedef struct {             /* gradient outputs, user order, float32 */
  int64_t n;                 /* rows of every buffer below; must equal the structure's n */
  float *means, *log_scales, *quats, *density, *sh;  /* [n,3] [n,3] [n,4] [n] [n,K,3] */
  float *sg;                 /* [n, n_sg, 7] lobe gradients, required when the structure has lobes */
  int32_t accumulate;        /* 0: overwrite, 1: add into the buffers */
  /* Densification statistic of Sec. 3.5 (Eq. 12), nullable: for each view v
     of the call, densify[i] += alpha_v |dL_v/dmu_i| with alpha_v =
     |mu_i - o_v| / f_v (o_v the camera centre, f_v = fx of view v) and
     L_v the loss restricted to view v's pixels; densify_views[i] += 1 when
     that gradient is non-zero.  Both are added to (never cleared), so the
     caller keeps the running sums between densification steps.  When
     densify is set the views are marched one at a time. */
  float *densify;            /* [n] */
  int32_t *densify_views;    /* [n], required with densify */
} rgx_grads;

/* per-ray statistics written by rgx_render_forward when `stats` is given */
enum {
  RGX_STAT_Q = 0,        /* distinct Gaussians in the hit sets of processed segments */
  RGX_STAT_P,            /* (segment, Gaussian) pairs over processed segments */
  RGX_STAT_SAMPLES,      /* samples evaluated (t < t_far, non-empty segments) */
  RGX_STAT_SEGMENTS,     /* non-empty segments processed */
  RGX_STAT_CLOSEST,      /* closest-hit queries */
  RGX_STAT_BOX_ONLY,     /* per ray, summed over its window collections: visited leaves whose
                            AABB meets the ray's window interval while the ellipsoid chord
                            does not (the AABB false positives) */
  RGX_STAT_NODES,        /* BVH nodes loaded by the wave for the segment collections */
  RGX_STAT_LEAVES,       /* leaves the wave visited for the segment collections */
  RGX_STAT_WINDOWS,      /* window collections the wave made (attempts included) */
  RGX_STAT_CHUNKED,      /* segments whose candidates were collected in several Z chunks */
  RGX_STAT_CAND,         /* per wave: candidates passing the window list's depth pre-checks
                            (the wave's span, then some lane's own segment) */
  RGX_STAT_CAND_HIT,     /* per wave: candidates that some lane hit */
  RGX_STAT_KCYC_COLLECT, /* per wave: shader-clock kilocycles in window collection */
  RGX_STAT_KCYC_CLOSEST, /* per wave: kilocycles in closest-hit queries */
  RGX_STAT_KCYC_TILE,    /* per wave: kilocycles for the whole tile */
  RGX_STAT_T_END,        /* float bits: where the ray's march ended (Alg. 1): the start of the
                            first segment with T <= T_eps, else t_far */
  RGX_NSTAT = 16
};

/* Totals of one forward's per-ray statistics, returned by rgx_sync_stats */
enum {
  RGX_TOT_RAYS = 0,      /* rays rendered */
  RGX_TOT_Q,             /* sum of RGX_STAT_Q */
  RGX_TOT_P,             /* sum of RGX_STAT_P */
  RGX_TOT_SAMPLES,       /* sum of RGX_STAT_SAMPLES */
  RGX_TOT_SEGMENTS,      /* sum of RGX_STAT_SEGMENTS */
  RGX_TOT_CLOSEST,       /* sum of RGX_STAT_CLOSEST */
  RGX_TOT_NODES,         /* BVH nodes loaded for window collections, summed over waves */
  RGX_TOT_BOX_ONLY,      /* sum of RGX_STAT_BOX_ONLY (AABB-only leaves per window collection) */
  RGX_TOT_CHUNKED,       /* segments whose window list overflowed and was taken in Z chunks */
  RGX_TOT_INACTIVE,      /* Gaussians of the structure that are inactive */
  RGX_TOT_UNRECORDED,    /* 64-ray tiles whose searches did not fit the state's record (their
                            backward searches again, with the same results) */
  RGX_NTOT = 11
};

/* Create / destroy a context on HIP device `device`.  rgx_create allocates. */
rgx_status rgx_create(int device, rgx_context **out);
void rgx_destroy(rgx_context *ctx);

/* Largest supported number of Gaussians (the marching kernels sort window
   lists on 32-bit keys that hold a 23-bit Z index). */
#define RGX_MAX_GAUSSIANS (1 << 23)

/* Build (or rebuild in place when *bvh is non-NULL) the acceleration
   structure: per-Gaussian preprocessing (R from the normalised quaternion,
   s = exp(l), M = S^-1 R^T, k^2 = 2 ln(sigma~/sigma_eps), minimal AABB
   half-lengths L_i = k sqrt(sum_j r_ij^2 s_j^2) padded outward, bounding
   sphere radius k max(s)), Morton keys of the means quantised over their
   bounds (Sec. 3.3), a stable radix sort, the Z-ordered pack and a Karras
   LBVH whose node boxes are range unions of the leaf boxes.  1 <= n <=
   RGX_MAX_GAUSSIANS (else RGX_ERR_INVALID_ARG / RGX_ERR_UNSUPPORTED).
   Allocates device memory when the structure must grow (never during stream
   capture).  The parameters are copied; the caller may change them
   afterwards. */
rgx_status rgx_build_bvh(rgx_context *ctx, const rgx_gaussians *g, const rgx_build_opts *opts,
                         rgx_bvh **bvh, hipStream_t stream);
void rgx_bvh_destroy(rgx_bvh *bvh);
/* (host) number of Gaussians and SH degree the structure was built from */
int64_t rgx_bvh_size(const rgx_bvh *bvh);

/* Forward render of n_views views (host array) through Algorithm 1.
   out_rgb [R,3] and out_T [R] with R = sum of width*height; `stats`
   (nullable) receives [R, RGX_NSTAT] int32 counters.

   state: NULL renders only (nothing is recorded; no backward can follow).
   Otherwise *state receives the forward state needed by rgx_render_backward:
   a new handle when *state is NULL, else the given handle is reused in place
   (its buffers grow when needed and are kept, so a forward with a reused
   handle can be captured into a graph once a first call has sized them).
   With empty-space skipping on (and the BVH in use) the state records each
   ray's first four closest-hit results (Alg. 1 ClosestHit, Eq. 4; 16 B per
   ray), every window list its tiles collected, and (unless
   opts->no_sample_record) each segment's per-sample sums of density and
   colour (Eq. 3; 128 B per ray segment at N_s = 8), in a pool of 48 KB per
   64-ray tile on average, twice that with the sums (three times at N_s =
   16); a tile that does not
   fit is not recorded and its backward searches and sums again, with the
   same results.  With `stats` given, the state
   also receives the totals that rgx_sync_stats returns.  Any number of states
   may be outstanding; each belongs to one forward at a time.  If the call
   fails after a new handle was made, *state still holds it: destroy it. */
rgx_status rgx_render_forward(rgx_context *ctx, const rgx_bvh *bvh, const rgx_camera *cams,
                              int32_t n_views, const rgx_render_opts *opts, float *out_rgb,
                              float *out_T, int32_t *stats, rgx_fwd **state, hipStream_t stream);

/* Backward of the forward that filled `state` (adjoint of Eq. 3 along
   Algorithm 1): given that forward's outputs (out_rgb, out_T exactly as
   returned) and dL/d(out_rgb) [R,3], dL/d(out_T) [R] (nullable), writes
   dL/d(parameters) in user order.  The cameras and options are the state's.
   The sample schedule, the ESS restarts and the truncation boundaries are
   treated as constants.  Segments are taken in the forward's deterministic
   order, the recorded closest hits, window lists and per-sample sums
   replayed; the transmittance before every sample is recomputed from those
   sums, and the colour still to come behind a sample is the final colour
   minus the running prefix.
   RGX_ERR_STATE when `bvh` is not the structure build the forward rendered
   (rebuilt or replaced since) or the state belongs to another context;
   RGX_ERR_INVALID_ARG when grads->n differs from the structure's n. */
rgx_status rgx_render_backward(rgx_context *ctx, const rgx_bvh *bvh, const rgx_fwd *state,
                               const float *out_rgb, const float *out_T, const float *grad_rgb,
                               const float *grad_T, const rgx_grads *grads, hipStream_t stream);

/* Releases a forward state and its device memory (NULL is a no-op).  The
   caller makes sure no enqueued or captured work still uses it. */
void rgx_fwd_destroy(rgx_fwd *state);

/* (host) Waits for `stream` (the one the state's forward ran on) and writes
   the totals of that forward's statistics, out[RGX_NTOT].  RGX_ERR_STATE when
   the forward was not given a `stats` buffer. */
rgx_status rgx_sync_stats(rgx_context *ctx, const rgx_fwd *state, int64_t *out,
                          hipStream_t stream);

/* AABB false positives along whole rays (Sec. 3.4, Eq. 6; minimal AABB of
   Supp. B): for the rays `pix` (row-major pixel indices of the single view
   `cam`), count[i] = the number of active Gaussians whose minimal AABB
   mu +/- L, L_j = k sqrt(sum_m r_jm^2 s_m^2), meets the ray over
   [t_near, t_end[i]] (slab test) while the ellipsoid's chord does not.
   t_end [n_rays] device float, e.g. RGX_STAT_T_END of a forward.  Counts
   int32 [n_rays] device.  A statistics path, not used by the renderer. */
rgx_status rgx_false_positives(rgx_context *ctx, const rgx_bvh *bvh, const rgx_camera *cam,
                               const int32_t *pix, int32_t n_rays, const float *t_end,
                               int32_t *count, hipStream_t stream);

/* Debug: per-ray hit sets.  For the rays `pix` (row-major pixel indices of
   the single view `cam`), records every (segment start, Gaussian) pair of
   every processed segment in processing order: seg_a [n_rays, cap] float,
   ids [n_rays, cap] int32 user-order Gaussian ids, count [n_rays] the number
   of pairs (entries beyond cap are counted but not written). */
rgx_status rgx_dump_hits(rgx_context *ctx, const rgx_bvh *bvh, const rgx_camera *cam,
                         const rgx_render_opts *opts, const int32_t *pix, int32_t n_rays,
                         int32_t cap, float *seg_a, int32_t *ids, int32_t *count,
                         hipStream_t stream);

/* Debug: copies of the build's internal arrays for structure checks
   (synchronises the stream).  Any output may be NULL.
     keys  [n] uint64 sorted Morton keys (inactive Gaussians last, key 2^(3*bits))
     perm  [n] int32  user index of the i-th Z-ordered Gaussian
     aabb  [n,6] float leaf boxes (lo xyz, hi xyz) in Z order
     nodes [max(n-1,1), 16] float internal nodes: left box lo/hi, right box lo/hi,
           children as int bits (>= 0 internal, < 0 leaf ~i, INT32_MIN none) in
           words 3 and 7, the node's first and last leaf index in words 11 and 15
     nodes4 [max(n-1,1), 36] float 4-wide records, one per binary internal
           node (row = its index; the walk from row 0 reaches those it needs):
           4 child boxes (lo xyz, hi xyz) in words 0..23, 4
           child links as int bits in words 24..27 (>= 0 a 4-wide record, < 0
           leaf ~i, INT32_MIN none), 4 (first, last) leaf ranges in 28..35
     n_active (host) number of active Gaussians. */
rgx_status rgx_bvh_debug(rgx_context *ctx, const rgx_bvh *bvh, uint64_t *keys, int32_t *perm,
                         float *aabb, float *nodes, float *nodes4, int64_t *n_active,
                         hipStream_t stream);

/* Debug: device-side error flag of the context (synchronises the stream).
   flags[0] != 0 means results are invalid.  Every flag guards a condition
   that a structure built by rgx_build_bvh and arguments the host checks
   accept cannot reach (the stacks are sized for the deepest possible tree,
   segment lengths are checked against the FP32 resolution at t_far, and
   list and record overflows are handled by chunking and re-searching): 1 a
   closest-hit stack overflowed, 2 a traversal visited more nodes than the
   tree has, 3 a malformed node, 4 a segment made no progress in FP32, 5 a
   broken window-list record, 6 a false-positive walk's stack overflowed. */
rgx_status rgx_error_flags(rgx_context *ctx, int32_t *flags /*host*/, hipStream_t stream);

/* Isotropic scale loss (Sec. 3.4, Eq. 8, with the volume-ratio bound of
   Eq. 7 / Eq. 9): for s = exp(log_scales[i]) the bound is
   r_i = 2/(pi sqrt 3) (sum_j s_ij^2)^(3/2) / prod_j s_ij, and
   L = (1/n) sum_i (max(r_i, r0) - r0).  Writes L to *loss (device float) and
   dL/d(log_scales) to grad [n,3] (device; accumulate != 0 adds into it).
   log_scales is [n,3] device float32, 1 <= n <= RGX_MAX_GAUSSIANS, r0 > 0.
   The reduction is deterministic.  Allocates a small per-context workspace
   the first time (and when n grows). */
rgx_status rgx_isotropic_loss(rgx_context *ctx, int64_t n, const float *log_scales, float r0,
                              float *loss, float *grad, int32_t accumulate, hipStream_t stream);

/* Allocation-free variant of rgx_isotropic_loss, for callers that cannot
   allocate device memory (code under stream capture, tight serving loops,
   harnesses that forbid allocation).  Same arguments, results and
   deterministic reduction; the per-block partial sums go to a fixed
   256 KB workspace per device (one double per 256 Gaussians for up to
   RGX_MAX_GAUSSIANS Gaussians), held from the first rgx_create on the device
   until the process ends.  Never allocates or frees.  n beyond the workspace
   returns RGX_ERR_INVALID_ARG.  Every call on a device shares that device's
   workspace: calls that overlap on one device (several streams or contexts)
   race and give undefined results; calls ordered on one stream are safe. */
rgx_status rgx_isotropic_loss_noalloc(rgx_context *ctx, int64_t n, const float *log_scales,
                                      float r0, float *loss, float *grad, int32_t accumulate,
                                      hipStream_t stream);

/* One parameter array of an Adam step (host struct). */
typedef struct {
  int64_t n;                 /* floats in the arrays, >= 0 */
  float *param;              /* [n] updated in place */
  const float *grad;         /* [n] */
  float *m, *v;              /* [n] first and second moments, zero before the first step */
  float lr;                  /* learning rate of this array */
} rgx_adam_group;

/* Adam (Kingma and Ba, 2015), the optimizer of the training workload (the
   per-step rebuild of Sec. 5 / Supp. F is rgx_build_bvh): advances the
   device step counter *step (int32, zero before the first step) by one, then
   for every element of every group m = b1 m + (1 - b1) g, v = b2 v + (1 - b2)
   g^2, p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), t the new
   count.  The counter lives on the device, so a captured step replays with
   the right bias corrections.  groups is a host array of n_groups >= 1. */
rgx_status rgx_adam_step(rgx_context *ctx, const rgx_adam_group *groups, int32_t n_groups,
                         int32_t *step, float beta1, float beta2, float eps, hipStream_t stream);

/* Optional kernel timing, for measurement.  While enabled, every launch made
   by rgx_build_bvh, rgx_render_forward and rgx_render_backward is bracketed
   by two HIP events recorded on the caller's stream (so the interval is that
   launch's duration on its own stream).  Do not enable it while a stream is
   being captured into a graph.  Enabling or disabling clears the record. */
enum {
  RGX_KERN_BUILD = 0,    /* the whole build sequence of one rgx_build_bvh */
  RGX_KERN_FORWARD,      /* one forward march launch (one per chunk of views) */
  RGX_KERN_BACKWARD,     /* one backward march launch */
  RGX_KERN_FINALIZE,     /* gradient chain rule + scatter to user order */
  RGX_NKERN = 4
};
rgx_status rgx_set_kernel_timing(rgx_context *ctx, int32_t enable);
/* Waits for the recorded events and returns, per RGX_KERN_* kind, the summed
   milliseconds ms[RGX_NKERN] and the number of launches launches[RGX_NKERN]
   (host arrays).  reset != 0 clears the record afterwards. */
rgx_status rgx_kernel_times(rgx_context *ctx, double *ms, int64_t *launches, int32_t reset);

/* (host) 1 if the context's last rgx_render_backward replayed its forward's
   recorded searches, 0 if the state held no record and it searched itself. */
int32_t rgx_backward_replayed(const rgx_context *ctx);

/* (host) Caps the record pool of every later forward given a state on this
   context at max_bytes (0: no cap beyond the default sizing, which is 96 KB
   per 64-ray tile at N_s <= 8, at least 64 MB, at most 16 GiB).  Tiles whose records do
   not fit are not recorded (RGX_TOT_UNRECORDED counts them) and their
   backward searches and sums again, with the same results, so a cap trades
   backward time for device memory and never changes results.
   RGX_ERR_INVALID_ARG for a negative max_bytes. */
rgx_status rgx_set_record_limit(rgx_context *ctx, int64_t max_bytes);

const char *rgx_status_string(rgx_status s);
const char *rgx_last_error(const rgx_context *ctx);

#ifdef __cplusplus
}
#endif
#endif /* RGX_H */

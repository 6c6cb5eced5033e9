// Forward and backward ray marching through the Gaussian field (Sec. 3.1
// Eq. 1-3; Sec. 3.2 Algorithm 1, Eq. 4-5).
//
// Execution model: one wave64 (one workgroup) owns one tile of 64 rays.  Each
// lane marches its ray segment by segment (Alg. 1).  Candidate Gaussians come
// from a per-wave window list: for a depth window covering one or more
// segments of every live lane, a node-parallel walk of the LBVH gathers the
// Gaussians that may meet the packet of rays in its windows, each with
// conservative depth bounds (see trav_run).  Every segment then runs over
// that list with a wave-uniform depth pre-check, so one BVH walk serves
// several segments and its memory latency is spread over 64 independent node
// fetches per round.  A window too large for the list is processed in Z-index
// chunks: the walk pauses when the list is full and resumes after the chunk.
// The geometry of 64 list entries is fetched at once, one entry per lane, and
// handed to each candidate with readlane; colour records are read at
// wave-uniform addresses through the scalar cache.  Closest-hit restarts
// beyond the window use a depth-first packet traversal, nearer child first.
//
// Every ray meets its Gaussians in Z-index order (window lists and their
// chunks are sorted, brute force counts up), whatever packet, window, tile
// shape or ray order is used; the images of all these variants are
// therefore bit-identical.
#include "common.hpp"
#include "internal.hpp"


namespace rgx {

constexpr float kInf = __builtin_huge_valf();
constexpr float kHalfLog2e = 0.72134752044448170f;  // log2(e) / 2

struct Ray {
  float ox, oy, oz;  // wave-uniform camera centre
  float dx, dy, dz;  // unit direction
  float ix, iy, iz;  // 1 / direction (components clamped away from 0)
};

__device__ __forceinline__ float safe_inv(float d) {
  const float a = fabsf(d) < 1e-20f ? copysignf(1e-20f, d) : d;
  return 1.0f / a;
}

// Slab test of a (padded) AABB over the lane's interval [lo, hi], with the
// box's parametric range widened by a few ulps (robust traversal).
__device__ __forceinline__ bool box_hit(float lx, float ly, float lz, float hx, float hy, float hz,
                                        const Ray &r, float lo, float hi) {
  const float tx0 = (lx - r.ox) * r.ix, tx1 = (hx - r.ox) * r.ix;
  const float ty0 = (ly - r.oy) * r.iy, ty1 = (hy - r.oy) * r.iy;
  const float tz0 = (lz - r.oz) * r.iz, tz1 = (hz - r.oz) * r.iz;
  float bmin = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fminf(tz0, tz1));
  float bmax = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fmaxf(tz0, tz1));
  bmin = fmaf(-fabsf(bmin), 1e-6f, bmin);
  bmax = fmaf(fabsf(bmax), 1e-6f, bmax);
  return fmaxf(bmin, lo) <= fminf(bmax, hi);
}

// Entry parameter of the box over [lo, hi] (same slab arithmetic as box_hit),
// or +inf when the box misses the interval.
__device__ __forceinline__ float box_entry(float lx, float ly, float lz, float hx, float hy,
                                           float hz, const Ray &r, float lo, float hi) {
  const float tx0 = (lx - r.ox) * r.ix, tx1 = (hx - r.ox) * r.ix;
  const float ty0 = (ly - r.oy) * r.iy, ty1 = (hy - r.oy) * r.iy;
  const float tz0 = (lz - r.oz) * r.iz, tz1 = (hz - r.oz) * r.iz;
  float bmin = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fminf(tz0, tz1));
  float bmax = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fmaxf(tz0, tz1));
  bmin = fmaf(-fabsf(bmin), 1e-6f, bmin);
  bmax = fmaf(fabsf(bmax), 1e-6f, bmax);
  const float e = fmaxf(bmin, lo);
  return e <= fminf(bmax, hi) ? e : kInf;
}

// Geometry of one Gaussian (wave-uniform, from the scalar cache).
struct Gauss {
  float mx, my, mz, k2;
  float m[9];
  float sig, l2sig, rad;   // rad: bounding-sphere radius of the ellipsoid
  float ox, oy, oz;        // the camera centre in the local frame, M (o - mu) (with_origin)
};

// Fills the local-frame camera centre (shared by every ray of a wave).
__device__ __forceinline__ Gauss with_origin(Gauss g, float ox, float oy, float oz) {
  const float ex = ox - g.mx, ey = oy - g.my, ez = oz - g.mz;
  g.ox = fmaf(g.m[0], ex, fmaf(g.m[1], ey, g.m[2] * ez));
  g.oy = fmaf(g.m[3], ex, fmaf(g.m[4], ey, g.m[5] * ez));
  g.oz = fmaf(g.m[6], ex, fmaf(g.m[7], ey, g.m[8] * ez));
  return g;
}

__device__ __forceinline__ Gauss load_gauss(const float *geom, int j) {
  cfloat4p p = as_const4(geom) + 4 * j;
  const vf4 a = p[0], b = p[1], c = p[2], d = p[3];
  Gauss g;
  g.mx = a.x; g.my = a.y; g.mz = a.z; g.k2 = a.w;
  g.m[0] = b.x; g.m[1] = b.y; g.m[2] = b.z; g.m[3] = b.w;
  g.m[4] = c.x; g.m[5] = c.y; g.m[6] = c.z; g.m[7] = c.w;
  g.m[8] = d.x; g.sig = d.y; g.l2sig = d.z; g.rad = d.w;
  return g;
}

// Ray / ellipsoid {q <= k^2}: q(t) = A (t - t*)^2 + h^2 about the point of
// closest approach; the chord is t* -/+ sqrt((k^2 - h^2) / A).
struct Chord {
  float A, ts, h2, tin, tout;
  bool exists;
};

// The ray in the Gaussian's local frame (g carries the origin, with_origin).
__device__ __forceinline__ void ray_local(const Gauss &g, const Ray &r, float &opx, float &opy,
                                          float &opz, float &dpx, float &dpy, float &dpz) {
  opx = g.ox;
  opy = g.oy;
  opz = g.oz;
  dpx = fmaf(g.m[0], r.dx, fmaf(g.m[1], r.dy, g.m[2] * r.dz));
  dpy = fmaf(g.m[3], r.dx, fmaf(g.m[4], r.dy, g.m[5] * r.dz));
  dpz = fmaf(g.m[6], r.dx, fmaf(g.m[7], r.dy, g.m[8] * r.dz));
}

__device__ __forceinline__ Chord chord(const Gauss &g, const Ray &r) {
  float opx, opy, opz, dpx, dpy, dpz;
  ray_local(g, r, opx, opy, opz, dpx, dpy, dpz);
  Chord c;
  c.A = fmaf(dpx, dpx, fmaf(dpy, dpy, dpz * dpz));
  const float B = fmaf(opx, dpx, fmaf(opy, dpy, opz * dpz));
  const float rA = __builtin_amdgcn_rcpf(c.A);
  c.ts = -B * rA;
  const float px = fmaf(c.ts, dpx, opx), py = fmaf(c.ts, dpy, opy), pz = fmaf(c.ts, dpz, opz);
  c.h2 = fmaf(px, px, fmaf(py, py, pz * pz));
  c.exists = c.h2 <= g.k2;
  const float w = __builtin_amdgcn_sqrtf(fmaxf(g.k2 - c.h2, 0.0f) * rA);
  c.tin = c.ts - w;
  c.tout = c.ts + w;
  return c;
}

// Colour of a Gaussian at the lane's direction: c = sum_m f_m Y_m.  Every
// colour record is kColFloats long whatever the degree (zero past 3 sh_k) and
// Y_m = 0 for m >= sh_k, so the record is read at fixed offsets, without
// branches, and the terms past the degree add exact zeros.  The record's
// three 64-byte scalar loads (colour_load) can be issued ahead of work that
// does not need them, so that their latency overlaps it (colour_eval).
struct ColRec {
  vf4 f[kColFloats / 4];
};

__device__ __forceinline__ ColRec colour_load(const float *col, int j) {
  cfloat4p p = as_const4(col) + (size_t)(kColFloats / 4) * j;
  ColRec c;
#pragma unroll
  for (int q = 0; q < kColFloats / 4; q++) c.f[q] = p[q];
  // a scheduling barrier: the compiler would otherwise place the loads
  // just before their first use, and their latency would not overlap the
  // caller's work between colour_load and colour_eval
  __builtin_amdgcn_sched_barrier(0);
  return c;
}

__device__ __forceinline__ void colour_eval(const ColRec &rc, const float *Y, float &cr, float &cg,
                                            float &cb) {
  float acc[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int q = 0; q < kColFloats / 4; q++) {
    const float fv[4] = {rc.f[q].x, rc.f[q].y, rc.f[q].z, rc.f[q].w};
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const int flat = 4 * q + e;
      acc[flat % 3] = fmaf(fv[e], Y[flat / 3], acc[flat % 3]);
    }
  }
  cr = acc[0]; cg = acc[1]; cb = acc[2];
}

__device__ __forceinline__ void colour(const float *col, int j, const float *Y, float &cr,
                                       float &cg, float &cb) {
  colour_eval(colour_load(col, j), Y, cr, cg, cb);
}

// Spherical-Gaussian lobes of Gaussian j added to the lane's colour:
// c += a_k exp(lambda_k (u_k.d - 1)) for the kMaxSg packed lobes (absent
// lobes have a = 0).  One lobe (two 16-byte scalar loads) per iteration, so
// the lobes do not all hold scalar registers at once.
__device__ __forceinline__ void sg_colour(const float *sg, int j, float dx, float dy, float dz,
                                          float &cr, float &cg, float &cb) {
  cfloat4p p = as_const4(sg) + (size_t)(kSgFloats / 4) * j;
#pragma unroll 1
  for (int k = 0; k < kMaxSg; k++) {
    const vf4 a = p[2 * k], u = p[2 * k + 1];
    const float cosang = fmaf(u.x, dx, fmaf(u.y, dy, u.z * dz));
    const float g = __builtin_amdgcn_exp2f(a.w * kLog2e * (cosang - 1.0f));
    cr = fmaf(a.x, g, cr);
    cg = fmaf(a.y, g, cg);
    cb = fmaf(a.z, g, cb);
  }
}

// Wave-uniform DFS stack, entry i held by lane i % 64 of s0 .. s4.  The
// closest-hit walk pushes at most 3 entries per 4-wide record on its current
// path (the record's unvisited children).  The records sit at binary internal
// nodes, each strictly deeper than the one before it on a path, and binary
// internal nodes lie at most 86 levels deep (the Karras split positions grow
// strictly down the tree over the 63-bit key extended by a 23-bit index), so
// a path meets at most 87 records and the stack never holds more than 261
// entries: 320 always suffice.
struct WaveStack {
  int s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0, sp = 0, lane = 0;
  __device__ __forceinline__ bool push(int v) {
    if (sp < 64) s0 = lane == sp ? v : s0;
    else if (sp < 128) s1 = lane == sp - 64 ? v : s1;
    else if (sp < 192) s2 = lane == sp - 128 ? v : s2;
    else if (sp < 256) s3 = lane == sp - 192 ? v : s3;
    else if (sp < 320) s4 = lane == sp - 256 ? v : s4;
    else return false;
    sp++;
    return true;
  }
  __device__ __forceinline__ int pop() {
    sp--;
    const int q = sp >> 6, l = sp & 63;
    return q == 0 ? __builtin_amdgcn_readlane(s0, l)
         : q == 1 ? __builtin_amdgcn_readlane(s1, l)
         : q == 2 ? __builtin_amdgcn_readlane(s2, l)
         : q == 3 ? __builtin_amdgcn_readlane(s3, l)
                  : __builtin_amdgcn_readlane(s4, l);
  }
};

// Ends the compiler's freedom to sink a load towards its first use: the
// value must be in registers here, so loads written together are issued
// together and waited for once (empty asm statements, no instruction).
// pin_loaded: a per-lane (vector) value; pin_uniform: a wave-uniform one
// from the scalar cache.
__device__ __forceinline__ void pin_loaded(const vf4 &x) {
  asm volatile("" : : "v"(x.x), "v"(x.y), "v"(x.z), "v"(x.w));
}
__device__ __forceinline__ void pin_uniform(float x) { asm volatile("" : : "s"(x)); }
__device__ __forceinline__ void pin_lane(uint32_t x) { asm volatile("" : : "v"(x)); }

// ---------------------------------------------------------------------------
// Work distribution: global tile index -> view, pixel, output ray.

struct Pixel {
  int view, px, py, ray;
  bool valid;
};

__device__ __forceinline__ Pixel tile_pixel(const ViewTable &vt, const MarchOpts &op, int w,
                                            int lane) {
  int v = 0;
  while (v + 1 < vt.n_views && vt.v[v + 1].tile_begin <= w) v++;
  const View &V = vt.v[v];
  const int t = w - V.tile_begin;
  Pixel p;
  p.view = v;
  if (op.ray_order == 0) {
    const int r = t * 64 + lane;
    p.valid = r < V.width * V.height;
    p.px = r % V.width;
    p.py = r / V.width;
  } else {
    const int code = V.tile_order[t];
    const int tx = code & 0xffff, ty = code >> 16;
    p.px = tx * op.tile_w + (lane & (op.tile_w - 1));
    p.py = ty * op.tile_h + (lane >> op.tile_w_log2);
    p.valid = p.px < V.width && p.py < V.height;
  }
  p.ray = V.ray_begin + p.py * V.width + p.px;
  return p;
}

// A wave-uniform value held in a vector register: the camera centre is read
// throughout the march, and scalar registers are the scarcer resource there.
__device__ __forceinline__ float in_vgpr(float x) {
  float y;
  asm volatile("v_mov_b32 %0, %1" : "=v"(y) : "s"(x));
  return y;
}

__device__ __forceinline__ Ray make_ray(const View &V, int px, int py) {
  Ray r;
  r.ox = in_vgpr(V.c2w[3]); r.oy = in_vgpr(V.c2w[7]); r.oz = in_vgpr(V.c2w[11]);
  const float u = ((float)px + 0.5f - V.cx) / V.fx;
  const float v = ((float)py + 0.5f - V.cy) / V.fy;
  float dx = fmaf(V.c2w[0], u, fmaf(V.c2w[1], v, V.c2w[2]));
  float dy = fmaf(V.c2w[4], u, fmaf(V.c2w[5], v, V.c2w[6]));
  float dz = fmaf(V.c2w[8], u, fmaf(V.c2w[9], v, V.c2w[10]));
  const float inv = rsqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
  r.dx = dx * inv; r.dy = dy * inv; r.dz = dz * inv;
  r.ix = safe_inv(r.dx); r.iy = safe_inv(r.dy); r.iz = safe_inv(r.dz);
  return r;
}

// Non-persistent launches: block b -> a contiguous run of tiles per XCD
// (blocks are dealt to the 8 XCDs round robin).
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb >> 3, rem = nb & 7, x = b & 7, rank = b >> 3;
  return x * q + min(x, rem) + rank;
}

// Persistent launches: 8 queues, one contiguous chunk of tiles each; a wave
// drains its home queue, then the others.  Returns -1 when all are empty.
__device__ __forceinline__ int pop_tile(int32_t *queue, int n_tiles, int home, int lane) {
  const int per = (n_tiles + 7) >> 3;
  for (int k = 0; k < 8; k++) {
    const int qi = (home + k) & 7;
    const int begin = qi * per;
    const int len = min(per, n_tiles - begin);
    if (len <= 0) continue;
    int got = 0;
    if (lane == 0) got = atomicAdd(&queue[qi], 1);
    got = uniform_int(got);
    if (got < len) return begin + got;
  }
  return -1;
}

// Midpoint sample positions of a segment, t_k = o + (i0 + k + 1/2) dt: on the
// fixed grid o = t_n and i0 = N_s * segment index, otherwise o = a, i0 = 0.
// Held as t_0 and dt, t_k = t_0 + k dt (two registers instead of N_s).
struct Samples {
  float t0, dt;
  __device__ __forceinline__ float t(int k) const { return fmaf((float)k, dt, t0); }
};

// Eq. 5 with d_i = a (unit direction from the camera centre).
__device__ __forceinline__ float adaptive_dt(const MarchOpts &op, float a, float T) {
  const float base = fmaxf(a * op.inv_beta, op.dt_min);
  const float v = base * __builtin_amdgcn_exp2f(-__builtin_amdgcn_logf(T) * (1.0f / 3.0f));
  return v < op.dt_max ? v : op.dt_max;
}

// Per-lane segment state shared by forward and backward.
struct SegState {
  bool alive, pending;
  int seg_i;
  float a, cl_lo;
};


// The N_S sample weights of one Gaussian for one lane:
// w_k = sigma~ exp(-q(t_k)/2) if q(t_k) <= k^2 else 0.  With t_k = t_0 + k dt
// and q(t) = A (t - t*)^2 + h^2, the exponent log2 sigma~ - q_k log2(e)/2 is
// a quadratic in the sample index, e_0 + k e_1 + k^2 e_2, so each sample
// costs two FMAs before its exp2; the truncation test q_k <= k^2 is the
// same quadratic against log2 sigma~ - k^2 log2(e)/2.
// With SKIP, returns the (wave-uniform) mask of samples that some active
// lane sees inside the Gaussian: the others have w_k = 0 in every lane, and
// callers may skip them (adding their zero terms would change nothing).  The
// forward gains from it; in the backward the extra branches cost more
// registers than they save.
template <int NS, bool SKIP = false>
__device__ __forceinline__ uint32_t sample_weights(const Gauss &g, const Chord &c,
                                                   const Samples &sp, float *w) {
  const float u0 = sp.t0 - c.ts;
  const float Au0 = c.A * u0;
  const float e0 = fmaf(-fmaf(Au0, u0, c.h2), kHalfLog2e, g.l2sig);
  const float e1 = -kHalfLog2e * (2.0f * Au0 * sp.dt);
  const float e2 = -kHalfLog2e * (c.A * sp.dt * sp.dt);
  const float e_min = fmaf(-g.k2, kHalfLog2e, g.l2sig);
  uint32_t live = 0;
#pragma unroll
  for (int k = 0; k < NS; k++) {
    const float x = k == 0 ? e0 : fmaf((float)(k * k), e2, fmaf((float)k, e1, e0));
    const bool in = x >= e_min;
    if (SKIP) {
      w[k] = 0.0f;
      if (ballot(in) != 0) {
        w[k] = in ? __builtin_amdgcn_exp2f(x) : 0.0f;
        live |= 1u << k;
      }
    } else {
      const float e = __builtin_amdgcn_exp2f(x);
      w[k] = in ? e : 0.0f;
    }
  }
  return SKIP ? live : (1u << NS) - 1u;
}

// Segment bounds [a, b], step and sample positions of a live lane.
template <int NS>
__device__ __forceinline__ bool segment(const MarchOpts &op, bool grid, const SegState &ss,
                                        float tn, float T, float &a, float &b, float &dt,
                                        Samples &sp) {
  a = grid ? fmaf((float)(ss.seg_i * NS), op.dt, tn) : ss.a;
  dt = op.adaptive ? adaptive_dt(op, a, T) : op.dt;
  b = grid ? fmaf((float)((ss.seg_i + 1) * NS), op.dt, tn) : fmaf((float)NS, dt, a);
  sp.t0 = grid ? fmaf((float)(ss.seg_i * NS) + 0.5f, dt, tn) : fmaf(0.5f, dt, a);
  sp.dt = dt;
  return b > a;
}

// Restart at a closest hit t: on the fixed grid the segment holding t (never
// going back), otherwise t itself.
__device__ __forceinline__ void restart_at(const MarchOpts &op, float tn, float dS, float t,
                                           SegState &ss) {
  if (!op.adaptive && op.ess == 1) ss.seg_i = max(ss.seg_i, (int)floorf((t - tn) / dS));
  else ss.a = t;
}

// Next segment after [a, b]: the following one, or after an empty segment
// with skipping on, the closest hit `best` (kInf: unknown here -> query).
__device__ __forceinline__ void step_after(const MarchOpts &op, bool grid, bool nonempty, float best,
                                           float tn, float dS, float b, SegState &ss) {
  if (grid) ss.seg_i += 1;
  else ss.a = b;
  if (nonempty || !op.ess) return;
  if (best < kInf) restart_at(op, tn, dS, best, ss);
  else { ss.pending = true; ss.cl_lo = b; }
}

// Cross-lane helpers (gfx950): v_permlane32_swap / v_permlane16_swap exchange
// halves / rows between two registers; DPP row and quad permutes.
__device__ __forceinline__ float swap32_sum(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap16_sum(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float uniform_lane(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
// In-row DPP permute of x; a lane with no valid source keeps `id`.
template <int CTRL>
__device__ __forceinline__ float dpp_or(float x, float id) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(id), __float_as_int(x), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}
// Minimum over the wave of values that are never negative (+inf allowed;
// -0 counts as 0), without LDS traffic: the bit patterns of such floats
// order as signed integers, so each in-row DPP permute (quad xor 1, quad
// xor 2, half-row mirror, row mirror) is one fused integer minimum, leaving
// each row's minimum in every lane of the row; the four rows are then read
// back.
__device__ __forceinline__ float wave_min_nonneg_dpp(float v) {
  int x = __float_as_int(v);
  x = min(x, __builtin_amdgcn_update_dpp(0x7fffffff, x, 0xb1, 0xf, 0xf, false));
  x = min(x, __builtin_amdgcn_update_dpp(0x7fffffff, x, 0x4e, 0xf, 0xf, false));
  x = min(x, __builtin_amdgcn_update_dpp(0x7fffffff, x, 0x141, 0xf, 0xf, false));
  x = min(x, __builtin_amdgcn_update_dpp(0x7fffffff, x, 0x140, 0xf, 0xf, false));
  const int a = min(__builtin_amdgcn_readlane(x, 0), __builtin_amdgcn_readlane(x, 16));
  const int b = min(__builtin_amdgcn_readlane(x, 32), __builtin_amdgcn_readlane(x, 48));
  return __int_as_float(min(a, b));
}


// One reduce-scatter stage over DPP partners: of 2H values per lane, the
// half picked by lane bit BIT is kept and the partner's other half added (the
// partner must differ from the lane in that bit).
template <int H, int CTRL, int BIT>
__device__ __forceinline__ void dpp_stage_bit(float *x, int lane) {
  const bool up = (lane & BIT) != 0;
#pragma unroll
  for (int i = 0; i < H; i++) {
    const float keep = up ? x[i + H] : x[i];
    const float send = up ? x[i] : x[i + H];
    x[i] = keep + dpp<CTRL>(send);
  }
}

// Sum over the wave of 16 per-lane slots.  Two half-wave swaps halve the
// slots per lane (lane bits 5 and 4 pick the half kept), two in-row DPP
// stages halve them again (bits 3 and 2, with the row and half-row mirrors
// as partners), and a quad sum completes the total.  Lane L returns the wave
// total of slot (L >> 2) & 15.
__device__ __forceinline__ float wave_sum_slots16(const float *g, int lane) {
  float y[8], z[4];
#pragma unroll
  for (int i = 0; i < 8; i++) y[i] = swap32_sum(g[i], g[i + 8]);
#pragma unroll
  for (int i = 0; i < 4; i++) z[i] = swap16_sum(y[i], y[i + 4]);
  dpp_stage_bit<2, 0x140, 8>(z, lane);   // row_mirror: lane p <-> 15 - p
  dpp_stage_bit<1, 0x141, 4>(z, lane);   // row_half_mirror: p <-> 7 - p within 8
  float u = z[0];
  u += dpp<0xb1>(u);                     // quad_perm [1,0,3,2]
  u += dpp<0x4e>(u);                     // quad_perm [2,3,0,1]
  return u;
}

// SH-coefficient gradients of a batch of up to 16 Gaussians, a small dense
// product on the matrix cores.  For Gaussian b of the batch and channel c,
// dL/df_{m,c} = sum over the tile's rays r of Y_m(d_r) G_c(r) S_b(r), S_b(r)
// the ray's sum over samples of w_k T_k phi_k (zero where the ray misses b).
// With A_c[m][r] = Y_m(d_r) G_c(r) fixed for the tile (held in registers)
// and B[r][b] = S_b(r) staged in LDS, each channel is 16 chained 16x16x4 FP32
// MFMAs over the 64 rays, computed transposed: D_c = B^T A_c^T, so that the
// result holds Gaussians in rows and coefficients in columns.  Operand
// layout of v_mfma_f32_16x16x4_f32 (wave64): first operand X[i][k] in lane
// i + 16k, second Y[k][j] in lane j + 16k, D[i][j] in lane j + 16 (i / 4),
// register i % 4.  Each atomic instruction therefore adds 16 consecutive
// floats (one 64-byte line) to each of 4 Gaussians' rows.
typedef float f4v __attribute__((ext_vector_type(4)));
constexpr int kSbStride = 66;   // floats per staged row: transposed reads hit distinct banks

struct ShBatch {
  float a[3][16];   // A_c for rays 4q + (lane >> 4), row m = lane & 15
  int n = 0;        // uniform: staged Gaussians
  int id = 0;       // lane b < 16: the Gaussian staged in row b
};

// A_c of a new tile; `tmp` is 192 floats of LDS free at that point.
__device__ __forceinline__ void sh_batch_start(ShBatch &B, float *sb, float *tmp, const float *Y,
                                               float g0, float g1, float g2, int lane) {
#pragma unroll
  for (int m = 0; m < 16; m++) sb[m * kSbStride + lane] = Y[m];
  tmp[lane] = g0;
  tmp[64 + lane] = g1;
  tmp[128 + lane] = g2;
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int q = 0; q < 16; q++) {
    const int ray = 4 * q + (lane >> 4);
    const float y = sb[(lane & 15) * kSbStride + ray];
    B.a[0][q] = y * tmp[ray];
    B.a[1][q] = y * tmp[64 + ray];
    B.a[2][q] = y * tmp[128 + ray];
  }
  __builtin_amdgcn_wave_barrier();
  B.n = 0;
}

// Multiplies out the staged batch and adds it to the accumulators.
__device__ __forceinline__ void sh_batch_flush(ShBatch &B, const float *sb, float *acc, int sh_k,
                                               int lane) {
  if (B.n == 0) return;
  __builtin_amdgcn_wave_barrier();
  f4v d0 = {0.0f, 0.0f, 0.0f, 0.0f}, d1 = d0, d2 = d0;
#pragma unroll
  for (int q = 0; q < 16; q++) {
    // S_b(r) for Gaussian b = lane & 15 and ray r = 4q + (lane >> 4)
    const float sv = sb[(lane & 15) * kSbStride + 4 * q + (lane >> 4)];
    d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(sv, B.a[0][q], d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(sv, B.a[1][q], d1, 0, 0, 0);
    d2 = __builtin_amdgcn_mfma_f32_16x16x4f32(sv, B.a[2][q], d2, 0, 0, 0);
  }
  // lane: coefficient m = lane & 15 of Gaussians 4 (lane >> 4) + i
  const int m = lane & 15;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const int b = 4 * (lane >> 4) + i;
    const int jb = __shfl(B.id, b, 64);
    if (b < B.n && m < sh_k) {
      float *row = acc + (size_t)kAccFloats * jb + 16;
      unsafeAtomicAdd(row + m, d0[i]);
      unsafeAtomicAdd(row + 16 + m, d1[i]);
      unsafeAtomicAdd(row + 32 + m, d2[i]);
    }
  }
  __builtin_amdgcn_wave_barrier();
  B.n = 0;
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return uniform_float(v);
}
// Wave minimum and maximum (exact, so the order of the reduction does not
// matter) without LDS traffic: four in-row DPP permutes (quad xor 1, quad
// xor 2, half-row mirror, row mirror) leave each row's extreme in every lane
// of the row, and the four rows are read out.  Called with the whole wave
// active.
__device__ __forceinline__ float wave_min(float v) {
  v = fminf(v, dpp_or<0xb1>(v, kInf));
  v = fminf(v, dpp_or<0x4e>(v, kInf));
  v = fminf(v, dpp_or<0x141>(v, kInf));
  v = fminf(v, dpp_or<0x140>(v, kInf));
  const float a = fminf(uniform_lane(v, 0), uniform_lane(v, 16));
  const float b = fminf(uniform_lane(v, 32), uniform_lane(v, 48));
  return fminf(a, b);
}
__device__ __forceinline__ float wave_max(float v) {
  v = fmaxf(v, dpp_or<0xb1>(v, -kInf));
  v = fmaxf(v, dpp_or<0x4e>(v, -kInf));
  v = fmaxf(v, dpp_or<0x141>(v, -kInf));
  v = fmaxf(v, dpp_or<0x140>(v, -kInf));
  const float a = fmaxf(uniform_lane(v, 0), uniform_lane(v, 16));
  const float b = fmaxf(uniform_lane(v, 32), uniform_lane(v, 48));
  return fmaxf(a, b);
}

// Closest hit (Alg. 1 ClosestHit, Eq. 4) for the lanes with `pending` set:
// min over Gaussians whose chord meets [cl_lo, t_far] of max(t_in, cl_lo).
// Depth-first packet traversal, nearer child first (by the smallest entry
// over the wave's pending lanes); each lane's bound shrinks to its best hit
// so far and prunes.  A minimum does not depend on the visiting order.
// Query qn of ray `ray`: recorded into (or, for q < kReplayK, replayed from)
// op.replay when op.replay_mode asks for it.
__device__ __forceinline__ void closest_pass(const SceneDev &s, const MarchOpts &op, int n_active,
                                             const Ray &r, float tn, float tf, float dS,
                                             SegState &ss, int32_t *err, int32_t *st_closest,
                                             int &qn, int64_t ray) {
  if (ballot(ss.pending) == 0) return;
  const bool replayed = op.replay_mode == 2 && ss.pending && qn < kReplayK;
  const float rbest = replayed ? op.replay[ray * kReplayK + qn] : kInf;
  const bool search = ss.pending && !replayed;
  const float lo = search ? ss.cl_lo : kInf;
  float hi = search ? tf : -kInf;
  float best = kInf;
  // Every candidate value max(t_in, lo) is at least lo: a lane whose best
  // reached lo has its answer and leaves the search (hi below lo), so that
  // the boxes around a ray starting inside ellipsoids are not all walked.
  auto leaf = [&](int j) {
    const Gauss g = with_origin(load_gauss(s.geom, j), r.ox, r.oy, r.oz);
    const Chord c = chord(g, r);
    if (c.exists && c.tin <= hi && c.tout >= lo) {
      best = fminf(best, fmaxf(c.tin, lo));
      hi = best <= lo ? -kInf : fminf(hi, best);
    }
  };
  __builtin_amdgcn_s_setprio(3);   // a dependent walk, as the collection's
  if (ballot(search) == 0) {
    // every pending lane replays
  } else if (op.brute_force) {
    for (int j = 0; j < n_active; j++) leaf(j);
  } else if (n_active > 0) {
    const int n_inner = n_active > 1 ? n_active - 1 : 1;
    WaveStack st;
    st.lane = __lane_id();
    st.sp = 0;
    int node = 0, visits = 0;
    for (;;) {
      if (ballot(hi >= lo) == 0) break;   // every searching lane has its answer
      if (node < 0) {
        if (st.sp == 0) break;
        const int v = st.pop();
        if (v < 0) { leaf(~v); continue; }
        node = v;
      }
      if (++visits > n_inner) { if (err) *err = 2; break; }
      cfloat4p np = as_const4(s.nodes4) + (kNode4Floats / 4) * node;
      float f[kNode4Floats];
#pragma unroll
      for (int q = 0; q < kNode4Floats / 4; q++) {
        const vf4 x = np[q];
        f[4 * q] = x.x; f[4 * q + 1] = x.y; f[4 * q + 2] = x.z; f[4 * q + 3] = x.w;
      }
      // the boxes and links go out as one batch of loads: the box tests and
      // the link checks below would otherwise each wait for a load of their
      // own
#pragma unroll
      for (int q = 0; q < 24 + 4; q++) pin_uniform(f[q]);
      int link[4];
      float e[4];
#pragma unroll
      for (int k = 0; k < 4; k++) {
        link[k] = __float_as_int(f[24 + k]);
        e[k] = link[k] != kNoChild
                   ? wave_min_nonneg_dpp(box_entry(f[6 * k], f[6 * k + 1], f[6 * k + 2], f[6 * k + 3],
                                                   f[6 * k + 4], f[6 * k + 5], r, lo, hi))
                   : kInf;
      }
      // links out of range (a malformed tree) end the walk; checked after
      // the box tests, which do not need them, in one branch-free test
      int bad = 0;
#pragma unroll
      for (int k = 0; k < 4; k++) {
        const int lk = link[k];
        bad |= (lk != kNoChild) & (lk >= 0 ? lk >= n_inner : ~lk >= n_active);
      }
      if (bad) { if (err) *err = 3; break; }
      // nearest child next; the others on the stack, farthest first (the
      // entries are wave-uniform, so this small sort is uniform too)
#pragma unroll
      for (int x = 0; x < 3; x++)
#pragma unroll
        for (int y = 0; y < 3 - x; y++)
          if (e[y + 1] < e[y]) {
            const float te = e[y]; e[y] = e[y + 1]; e[y + 1] = te;
            const int tl = link[y]; link[y] = link[y + 1]; link[y + 1] = tl;
          }
      bool overflow = false;
#pragma unroll
      for (int k = 3; k >= 1; k--)
        if (e[k] < kInf && !st.push(link[k])) overflow = true;
      if (overflow) { if (err) *err = 1; break; }
      if (!(e[0] < kInf)) { node = -1; continue; }
      if (link[0] >= 0) node = link[0];
      else { leaf(~link[0]); node = -1; }
    }
  }
  __builtin_amdgcn_s_setprio(0);
  if (ss.pending) {
    if (replayed) best = rbest;
    else if (op.replay_mode == 1 && qn < kReplayK) op.replay[ray * kReplayK + qn] = best;
    qn++;
    if (st_closest) (*st_closest)++;
    if (!(best < kInf)) ss.alive = false;
    else restart_at(op, tn, dS, best, ss);
    ss.pending = false;
  }
}

// ---------------------------------------------------------------------------
// Window collection.  For a per-lane depth window [lo, hi] the wave gathers
// every Gaussian that may meet some lane's window, restricted to the Z-index
// range [z0, z1), with a conservative depth interval for each.  Every test is
// against the packet as a whole: the bounding cone of the rays (apex at the
// shared camera centre) and the shell between the nearest window start and
// the farthest window end, applied to bounding spheres (of a node's child
// boxes, of a leaf's ellipsoid).  Exact per-ray chords are left to the
// segment loop, which computes them anyway.  The traversal is node-parallel:
// the frontier of (node, first leaf) is an LDS stack ordered by first leaf,
// smallest on top; each round hands the (up to) 64 lowest subtrees to the 64
// lanes, which load them independently, and their children go back on top in
// order -- a 64-wide depth-first walk in Z order, whose frontier stays narrow.
// When
// the frontier or the list would overflow, z1 is lowered (a radix select over
// the pending Z indices) and everything at or beyond it is dropped, so the
// result is always complete for [z0, z1); the caller continues from z1 with
// another chunk.  The list is finally sorted by Z index, so every ray meets
// its Gaussians in Z order whatever window, chunking or packet produced the
// list -- the order of brute force.

constexpr int kRingCap = 256;    // frontier (stack) entries
constexpr int kStageCap = 160;   // staged leaves; a round adds at most 2 per node
constexpr int kListCap = 512;    // window list entries (multiple of 64, at most 512)

struct WaveMem {
  float rdx[64], rdy[64], rdz[64], rix[64], riy[64], riz[64], rlo[64], rhi[64];
  struct {                         // traversal state, kept while a collection is paused
    int32_t ring_id[kRingCap], ring_first[kRingCap];
    int32_t st_id[kStageCap];
  } c;
  int32_t order[kListCap];         // slots of the current chunk's entries, in Z-index order
  int32_t l_id[kListCap];
  float l_tin[kListCap], l_tout[kListCap];
  int32_t cnt_box[64];             // per-ray AABB-only leaf count (statistics)
};

__device__ __forceinline__ uint64_t join64(uint32_t lo, uint32_t hi) {
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

__device__ __forceinline__ uint64_t lanes_below(int lane) {
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Lane-local ray r from the wave's LDS copy (origin is wave-uniform).
__device__ __forceinline__ Ray lds_ray(const WaveMem &M, const Ray &self, int r) {
  Ray q;
  q.ox = self.ox; q.oy = self.oy; q.oz = self.oz;
  q.dx = M.rdx[r]; q.dy = M.rdy[r]; q.dz = M.rdz[r];
  q.ix = M.rix[r]; q.iy = M.riy[r]; q.iz = M.riz[r];
  return q;
}

// Loads one geometry record at a per-lane address (vector memory path).
__device__ __forceinline__ Gauss load_gauss_lane(const float *geom, int j) {
  const vf4 *p = reinterpret_cast<const vf4 *>(geom) + 4 * j;
  const vf4 a = p[0], b = p[1], c = p[2], d = p[3];
  Gauss g;
  g.mx = a.x; g.my = a.y; g.mz = a.z; g.k2 = a.w;
  g.m[0] = b.x; g.m[1] = b.y; g.m[2] = b.z; g.m[3] = b.w;
  g.m[4] = c.x; g.m[5] = c.y; g.m[6] = c.z; g.m[7] = c.w;
  g.m[8] = d.x; g.sig = d.y; g.l2sig = d.z; g.rad = d.w;
  return g;
}

// Largest z in [zlo, zhi] such that at most `target` of the wave's values
// (V per lane, where ok) are below z.  zlo, zhi and the result are uniform.
template <int V>
__device__ __forceinline__ int select_cut(const int (&v)[V], const bool (&ok)[V], int zlo, int zhi,
                                          int target) {
  while (zlo < zhi) {
    const int mid = zlo + ((zhi - zlo + 1) >> 1);
    int c = 0;
#pragma unroll
    for (int k = 0; k < V; k++) c += __popcll(ballot(ok[k] && v[k] < mid));
    if (c <= target) zlo = mid;
    else zhi = mid - 1;
  }
  return zlo;
}

// Keeps the list entries with index < z1 (order preserved); returns the
// count.  64 entries at a time: a write never passes an unread entry.
__device__ __forceinline__ int compact_list(WaveMem &M, int lane, int count, int z1) {
  const uint64_t below = lanes_below(lane);
  int base = 0;
  for (int e0 = 0; e0 < count; e0 += 64) {
    const int e = e0 + lane;
    int id = 0;
    float tin = 0.0f, tout = 0.0f;
    bool keep = false;
    if (e < count) {
      id = M.l_id[e];
      tin = M.l_tin[e];
      tout = M.l_tout[e];
      keep = id < z1;
    }
    __builtin_amdgcn_wave_barrier();
    const uint64_t b = ballot(keep);
    if (keep) {
      const int pos = base + __popcll(b & below);
      M.l_id[pos] = id;
      M.l_tin[pos] = tin;
      M.l_tout[pos] = tout;
    }
    base += __popcll(b);
    __builtin_amdgcn_wave_barrier();
  }
  return base;
}

// Keeps the frontier entries in [head, tail) whose first leaf is below z1
// (order preserved, same scheme); returns the new end.
__device__ __forceinline__ int compact_ring(WaveMem &M, int lane, int head, int tail, int z1) {
  const uint64_t below = lanes_below(lane);
  int base = head;
  for (int e0 = head; e0 < tail; e0 += 64) {
    const int e = e0 + lane;
    const int slot = e;
    int id = 0, first = 0;
    bool keep = false;
    if (e < tail) {
      id = M.c.ring_id[slot];
      first = M.c.ring_first[slot];
      keep = first < z1;
    }
    __builtin_amdgcn_wave_barrier();
    const uint64_t b = ballot(keep);
    if (keep) {
      const int d = base + __popcll(b & below);
      M.c.ring_id[d] = id;
      M.c.ring_first[d] = first;
    }
    base += __popcll(b);
    __builtin_amdgcn_wave_barrier();
  }
  return base;
}

// In-lane stage of the register bitonic sort: element 64q + lane is paired
// with 64(q ^ JQ) + lane (the same lane).
template <int JQ>
__device__ __forceinline__ void bitonic_inlane(uint32_t (&key)[8], int k, int nq) {
#pragma unroll
  for (int q = 0; q < 8; q++) {
    const int p = q ^ JQ;
    if (p > q && p < nq) {
      const bool up = ((64 * q) & k) == 0;
      const uint32_t x = key[q], y = key[p];
      const uint32_t lo = x < y ? x : y, hi = x < y ? y : x;
      key[q] = up ? lo : hi;
      key[p] = up ? hi : lo;
    }
  }
}

// Orders the list entries with index below zc by Gaussian (Z) index (the
// other entries stay in the list for a later chunk): the keys (index << 9 |
// slot; indices are distinct and below 2^23) are sorted by a bitonic network
// held in registers, element 64q + lane in key[q] -- partners in other lanes
// are read with cross-lane shuffles, partners in the same lane are registers.
// The sorted slots go to M.order.  Returns how many there are.
__device__ __forceinline__ int sort_list(WaveMem &M, int lane, int count, int zc) {
  static_assert(kListCap <= 512, "sort keys hold a 9-bit slot");
  int p2 = 64;
  while (p2 < count) p2 <<= 1;
  const int nq = p2 >> 6;
  uint32_t key[8];
  int valid = 0;
#pragma unroll
  for (int q = 0; q < 8; q++) {
    const int e = 64 * q + lane;
    const int id = e < count ? M.l_id[e] : 0x7fffffff;
    key[q] = id < zc ? ((uint32_t)id << 9) | (uint32_t)e : 0xffffffffu;
    valid += __popcll(ballot(id < zc));
  }
  for (int k = 2; k <= p2; k <<= 1) {
    for (int j = k >> 1; j >= 1; j >>= 1) {
      if (j >= 64) {
        if (j == 64) bitonic_inlane<1>(key, k, nq);
        else if (j == 128) bitonic_inlane<2>(key, k, nq);
        else bitonic_inlane<4>(key, k, nq);
      } else {
        const bool lower = (lane & j) == 0;
#pragma unroll
        for (int q = 0; q < 8; q++) {
          if (q < nq) {
            const uint32_t x = key[q];
            const uint32_t y = (uint32_t)__shfl_xor((int)x, j, 64);
            const bool up = ((64 * q + lane) & k) == 0;
            const uint32_t lo = x < y ? x : y, hi = x < y ? y : x;
            key[q] = up == lower ? lo : hi;
          }
        }
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int q = 0; q < 8; q++) {
    const int e = 64 * q + lane;
    if (e < valid) M.order[e] = (int)(key[q] & 511u);
  }
  __builtin_amdgcn_wave_barrier();
  return valid;
}

// The packet bound: apex o, unit axis u, half-angle (cos, sin) padded
// outward, and the depth shell [t_lo, t_hi] (distances from o).
struct Cone {
  float ux, uy, uz, cs, sn, t_lo, t_hi;
  bool narrow;   // false: rays spread too far for the angular test
};

__device__ __forceinline__ Cone packet_cone(const WaveMem &M, const Ray &self, int lane,
                                            uint64_t rays) {
  const bool mine = (rays >> lane) & 1;
  const float sx = wave_sum_f(mine ? self.dx : 0.0f), sy = wave_sum_f(mine ? self.dy : 0.0f),
              sz = wave_sum_f(mine ? self.dz : 0.0f);
  Cone k;
  const float n2 = fmaf(sx, sx, fmaf(sy, sy, sz * sz));
  const float inv = n2 > 0.0f ? rsqrtf(n2) : 0.0f;
  k.ux = sx * inv; k.uy = sy * inv; k.uz = sz * inv;
  // sine and cosine of each ray's angle to the axis (cross product: no
  // cancellation at small angles)
  const float cx = self.dy * k.uz - self.dz * k.uy, cy = self.dz * k.ux - self.dx * k.uz,
              cz = self.dx * k.uy - self.dy * k.ux;
  const float sn = wave_max(mine ? sqrtf(fmaf(cx, cx, fmaf(cy, cy, cz * cz))) : 0.0f);
  const float cs = wave_min(mine ? fmaf(self.dx, k.ux, fmaf(self.dy, k.uy, self.dz * k.uz)) : 1.0f);
  k.narrow = n2 > 0.0f && cs > 0.5f;
  k.sn = fminf(sn * 1.0001f + 2e-6f, 1.0f);
  k.cs = sqrtf(fmaxf(1.0f - k.sn * k.sn, 0.0f));
  k.t_lo = wave_min(mine ? M.rlo[lane] : kInf);
  k.t_hi = wave_max(mine ? M.rhi[lane] : -kInf);
  return k;
}

// Conservative: false only if no point of the sphere (centre v relative to
// the apex, radius rho) lies on a ray of the packet at a depth inside the
// shell.  On true, [*dlo, *dhi] bounds the depth of every such point.
__device__ __forceinline__ bool cone_sphere(const Cone &k, float vx, float vy, float vz, float rho,
                                            float *dlo, float *dhi) {
  const float d = sqrtf(fmaf(vx, vx, fmaf(vy, vy, vz * vz)));
  // rho's margin covers the FP32 chord ends near tangency (~3e-4 of the extent)
  const float pad = fmaf(d, 1e-5f, rho * 1.001f);
  *dlo = d - pad;
  *dhi = d + pad;
  if (*dlo > k.t_hi || *dhi < k.t_lo) return false;
  const float al = fmaf(vx, k.ux, fmaf(vy, k.uy, vz * k.uz));
  if (al + pad < 0.0f) return false;
  if (!k.narrow) return true;
  const float wx = vy * k.uz - vz * k.uy, wy = vz * k.ux - vx * k.uz, wz = vx * k.uy - vy * k.ux;
  const float perp = sqrtf(fmaf(wx, wx, fmaf(wy, wy, wz * wz)));
  return fmaf(perp, k.cs, -al * k.sn) <= pad;
}

// Conservative test of an AABB against the packet, on the box itself: the
// depth shell through the box's exact distance range from the apex; the cone
// through the box's extent across and along the axis (every box point p has
// |p_perp| >= |c_perp| - r_w and p.u <= c.u + r_u, r_w and r_u the box's
// supports along the unit perpendicular of its centre and along the axis).
__device__ __forceinline__ bool cone_box(const Cone &k, const Ray &o, float lx, float ly, float lz,
                                         float hx, float hy, float hz) {
  const float cx = fmaf(0.5f, lx + hx, -o.ox), cy = fmaf(0.5f, ly + hy, -o.oy),
              cz = fmaf(0.5f, lz + hz, -o.oz);
  const float ex = 0.5f * (hx - lx), ey = 0.5f * (hy - ly), ez = 0.5f * (hz - lz);
  const float ax = fabsf(cx), ay = fabsf(cy), az = fabsf(cz);
  const float qx = fmaxf(ax - ex, 0.0f), qy = fmaxf(ay - ey, 0.0f), qz = fmaxf(az - ez, 0.0f);
  const float fx = ax + ex, fy = ay + ey, fz = az + ez;
  const float dmin = sqrtf(fmaf(qx, qx, fmaf(qy, qy, qz * qz)));
  const float dmax = sqrtf(fmaf(fx, fx, fmaf(fy, fy, fz * fz)));
  const float pad = fmaf(dmax, 2e-5f, 1e-6f);
  if (dmin - pad > k.t_hi || dmax + pad < k.t_lo) return false;
  const float al = fmaf(cx, k.ux, fmaf(cy, k.uy, cz * k.uz));
  const float ru = fmaf(ex, fabsf(k.ux), fmaf(ey, fabsf(k.uy), ez * fabsf(k.uz)));
  if (al + ru + pad < 0.0f) return false;
  if (!k.narrow) return true;
  const float wx = cy * k.uz - cz * k.uy, wy = cz * k.ux - cx * k.uz, wz = cx * k.uy - cy * k.ux;
  const float pw = sqrtf(fmaf(wx, wx, fmaf(wy, wy, wz * wz)));
  // unit perpendicular of the centre: c - (c.u) u, normalised by |c x u|
  const float px = fmaf(-al, k.ux, cx), py = fmaf(-al, k.uy, cy), pz = fmaf(-al, k.uz, cz);
  const float rw = fmaf(ex, fabsf(px), fmaf(ey, fabsf(py), ez * fabsf(pz))) *
                   __builtin_amdgcn_rcpf(fmaxf(pw, 1e-30f));
  // margins: 1e-3 of the box extent for the rounding of the perpendicular
  // direction, 2e-5 of the distance for the rest
  const float slack = fmaf(rw, 1e-3f, pad);
  return fmaf(pw - rw, k.cs, -(al + ru) * k.sn) <= slack;
}

// Depth bounds [lo, hi] of every ray of the packet inside one ellipsoid, and
// whether the ellipsoid can meet the cone at all (returned)
// (centre v relative to the apex, size k, scales s, unit quaternion q): a
// point o + t d of the ellipsoid satisfies |t - v.d| <= k |S R^T d| (its
// support along d), v.d ranges over [|v| cos(phi + theta), |v| cos(phi - theta)]
// for the angle phi between v and the axis, and |S R^T d| <= |S R^T u| +
// max(s) |d - u| with |d - u| <= sin(theta) sqrt(2 / (1 + cos(theta))).
__device__ __forceinline__ bool support_bounds(const Cone &k, float vx, float vy, float vz,
                                               float kk, float sx, float sy, float sz, float qw,
                                               float qx, float qy, float qz, float *lo,
                                               float *hi) {
  // w = R^T u, R the rotation of the unit quaternion
  const float R00 = 1.0f - 2.0f * (qy * qy + qz * qz), R01 = 2.0f * (qx * qy - qw * qz),
              R02 = 2.0f * (qx * qz + qw * qy);
  const float R10 = 2.0f * (qx * qy + qw * qz), R11 = 1.0f - 2.0f * (qx * qx + qz * qz),
              R12 = 2.0f * (qy * qz - qw * qx);
  const float R20 = 2.0f * (qx * qz - qw * qy), R21 = 2.0f * (qy * qz + qw * qx),
              R22 = 1.0f - 2.0f * (qx * qx + qy * qy);
  const float w0 = sx * fmaf(R00, k.ux, fmaf(R10, k.uy, R20 * k.uz));
  const float w1 = sy * fmaf(R01, k.ux, fmaf(R11, k.uy, R21 * k.uz));
  const float w2 = sz * fmaf(R02, k.ux, fmaf(R12, k.uy, R22 * k.uz));
  const float du = k.sn * sqrtf(2.0f / (1.0f + k.cs));
  const float ext = kk * fmaf(fmaxf(sx, fmaxf(sy, sz)), du, sqrtf(fmaf(w0, w0, fmaf(w1, w1, w2 * w2))));
  const float d = sqrtf(fmaf(vx, vx, fmaf(vy, vy, vz * vz)));
  const float al = fmaf(vx, k.ux, fmaf(vy, k.uy, vz * k.uz));
  const float cx = vy * k.uz - vz * k.uy, cy = vz * k.ux - vx * k.uz, cz = vx * k.uy - vy * k.ux;
  const float perp = sqrtf(fmaf(cx, cx, fmaf(cy, cy, cz * cz)));
  // phi >= theta <=> perp cos(theta) >= al sin(theta); phi <= 90 deg <=> al >= 0
  const float c_hi = perp * k.cs >= al * k.sn ? fmaf(al, k.cs, perp * k.sn) : d;
  const float c_lo = al >= 0.0f ? fmaf(al, k.cs, -perp * k.sn) : -d;
  // margins: FP32 chord ends near tangency, rotation and norm rounding
  const float pad = fmaf(ext, 1e-3f, fmaf(d, 1e-5f, 1e-6f));
  *lo = c_lo - ext - pad;
  *hi = c_hi + ext + pad;
  // the cone: every point p of the ellipsoid has |p_perp| >= perp - r_w and
  // p.u <= al + r_u, with r_w, r_u its supports along the unit perpendicular
  // of the centre and along the axis
  if (!(perp > 0.0f)) return true;
  const float ip = __builtin_amdgcn_rcpf(perp);
  const float px = fmaf(-al, k.ux, vx) * ip, py = fmaf(-al, k.uy, vy) * ip,
              pz = fmaf(-al, k.uz, vz) * ip;
  const float y0 = sx * fmaf(R00, px, fmaf(R10, py, R20 * pz));
  const float y1 = sy * fmaf(R01, px, fmaf(R11, py, R21 * pz));
  const float y2 = sz * fmaf(R02, px, fmaf(R12, py, R22 * pz));
  const float rw = kk * sqrtf(fmaf(y0, y0, fmaf(y1, y1, y2 * y2)));
  const float ru = kk * sqrtf(fmaf(w0, w0, fmaf(w1, w1, w2 * w2)));
  const float slack = fmaf(rw + ru, 1e-3f, fmaf(d, 2e-5f, 1e-6f));
  return fmaf(perp - rw, k.cs, -(al + ru) * k.sn) <= slack;
}

// Wave-uniform state of a window collection.  The list holds the entries
// found so far; the frontier stack and the staged leaves live in M.c.  A
// collection ends either complete for [z0, z1) (z1 may have been lowered by a
// cut) or paused: the list is full, and its entries below zp -- everything
// below the smallest pending Z index -- form a complete chunk [z0, zp); after
// that chunk, trav_advance drops those entries and trav_run resumes.
struct Trav {
  uint64_t rays;                   // lanes whose windows (M.rlo, M.rhi) are collected
  int z0, z1, zp;
  int sp, staged, count, visits;
  bool paused;
};

__device__ __forceinline__ void trav_start(WaveMem &M, int lane, Trav &t, uint64_t rays, int z0,
                                           int z1) {
  t.rays = rays;
  t.z0 = z0;
  t.z1 = z1;
  t.zp = z1;
  t.sp = 1;
  t.staged = 0;
  t.count = 0;
  t.visits = 0;
  t.paused = false;
  if (lane == 0) {
    M.c.ring_id[0] = 0;
    M.c.ring_first[0] = 0;
  }
  __builtin_amdgcn_wave_barrier();
}

// Drops the entries of a finished chunk [z0, zp) and moves z0 to zp.
__device__ __forceinline__ void trav_advance(WaveMem &M, int lane, Trav &t) {
  const uint64_t below = lanes_below(lane);
  int base = 0;
  for (int e0 = 0; e0 < t.count; e0 += 64) {
    const int e = e0 + lane;
    int id = 0;
    float tin = 0.0f, tout = 0.0f;
    bool keep = false;
    if (e < t.count) {
      id = M.l_id[e];
      tin = M.l_tin[e];
      tout = M.l_tout[e];
      keep = id >= t.zp;
    }
    __builtin_amdgcn_wave_barrier();
    const uint64_t b = ballot(keep);
    if (keep) {
      const int pos = base + __popcll(b & below);
      M.l_id[pos] = id;
      M.l_tin[pos] = tin;
      M.l_tout[pos] = tout;
    }
    base += __popcll(b);
    __builtin_amdgcn_wave_barrier();
  }
  t.count = base;
  t.z0 = t.zp;
  t.zp = t.z1;
  t.paused = false;
}

// Runs (or resumes) the collection until it completes or pauses; sorts the
// finished chunk's entries into M.order and returns their number, or -1 on
// a malformed tree (error flag set).
__device__ __forceinline__ int trav_run(const SceneDev &s, WaveMem &M, const Ray &self, int lane, Trav &t,
                        int n_active, bool stats, int32_t *err, int32_t &nodes_out,
                        int32_t &leaves_out, int64_t *cyc_excl) {
  if (n_active <= 0 || t.rays == 0 || t.z0 >= t.z1) {
    t.count = 0;
    t.sp = 0;
    t.staged = 0;
    return 0;
  }
  const int n_inner = n_active > 1 ? n_active - 1 : 1;
  const uint64_t rays = t.rays;
  const int z0 = t.z0;
  int z1 = t.z1;
  // stack S[0, sp): first leaf strictly decreasing towards the top S[sp-1]
  int sp = t.sp, staged = t.staged, count = t.count, visits = t.visits;
  const int visits0 = visits;
  const Cone cone = packet_cone(M, self, lane, rays);
  const uint64_t below = lanes_below(lane);
  for (;;) {
    __builtin_amdgcn_wave_barrier();
    const int n = min(min(64, sp), (kStageCap - staged) >> 1);
    if (n > 0) {
      int id = 0;
      bool live = false;
      if (lane < n) {                            // lane 0 takes the top (lowest Z)
        const int slot = sp - 1 - lane;
        id = M.c.ring_id[slot];
        live = M.c.ring_first[slot] < z1;      // else cut off by a later z1
      }
      sp -= n;
      visits += __popcll(ballot(live));
      if (visits > n_inner) { if (err) *err = 2; t.count = 0; t.sp = 0; t.staged = 0; return -1; }
      vf4 a = {0, 0, 0, 0}, b = {0, 0, 0, 0}, c = {0, 0, 0, 0}, d = {0, 0, 0, 0};
      if (live) {
        const vf4 *np = reinterpret_cast<const vf4 *>(s.nodes) + 4 * id;
        a = np[0]; b = np[1]; c = np[2]; d = np[3];
      }
      const int cl = live ? __float_as_int(a.w) : kNoChild;
      const int cr = live ? __float_as_int(b.w) : kNoChild;
      const int nlo = __float_as_int(c.w), nhi = __float_as_int(d.w);
      const int gamma = cl < 0 ? ~cl : cl;       // left range [nlo, gamma], right [gamma+1, nhi]
      // validity of the links and ranges (a malformed tree ends the walk),
      // then the Z-range and packet tests: plain conjunctions, so that they
      // stay in lane masks instead of branching on every term
      const bool badL = cl >= 0 ? cl >= n_inner : ~cl >= n_active;
      const bool badR = (cr != kNoChild) &
                        ((cr >= 0 ? cr >= n_inner : ~cr >= n_active) |
                         !((0 <= nlo) & (nlo <= gamma) & (gamma < nhi) & (nhi < n_active)));
      const bool bad = live & (badL | badR);
      if (ballot(bad)) { if (err) *err = 3; t.count = 0; t.sp = 0; t.staged = 0; return -1; }
      const bool inL = live & (nlo < z1) & (gamma >= z0);
      const bool inR = live & (cr != kNoChild) & (gamma + 1 < z1) & (nhi >= z0);
      const bool hL = inL & cone_box(cone, self, a.x, a.y, a.z, b.x, b.y, b.z);
      const bool hR = inR & cone_box(cone, self, c.x, c.y, c.z, d.x, d.y, d.z);
      // children, in lane order, left before right
      bool lI = hL && cl >= 0, rI = hR && cr >= 0;
      const bool lL = hL && cl < 0, rL = hR && cr < 0;
      {
        int tot = __popcll(ballot(lI)) + __popcll(ballot(rI));
        if (sp + tot > kRingCap) {
          // frontier overflow: lower z1 to keep half the pending subtrees
          int v[kRingCap / 64 + 2];
          bool ok[kRingCap / 64 + 2];
#pragma unroll
          for (int k = 0; k < kRingCap / 64; k++) {
            const int e = lane + 64 * k;
            ok[k] = e < sp;
            v[k] = ok[k] ? M.c.ring_first[e] : 0;
          }
          v[kRingCap / 64] = nlo; ok[kRingCap / 64] = lI;
          v[kRingCap / 64 + 1] = gamma + 1; ok[kRingCap / 64 + 1] = rI;
          z1 = select_cut(v, ok, z0 + 1, z1, kRingCap / 2);
          sp = compact_ring(M, lane, 0, sp, z1);
          lI = lI && nlo < z1;
          rI = rI && gamma + 1 < z1;
          tot = __popcll(ballot(lI)) + __popcll(ballot(rI));
        }
        // the children are below every entry left on the stack; in lane
        // order, left before right, they are ascending, so the k-th of them
        // goes to S[sp + tot - 1 - k]
        const uint64_t b1 = ballot(lI || rI), b2 = ballot(lI && rI);
        const int rank = __popcll(b1 & below) + __popcll(b2 & below);
        int pos = sp + tot - 1 - rank;
        if (lI) {
          M.c.ring_id[pos] = cl;
          M.c.ring_first[pos] = nlo;
          pos--;
        }
        if (rI) {
          M.c.ring_id[pos] = cr;
          M.c.ring_first[pos] = gamma + 1;
        }
        sp += tot;
      }
      {
        // leaves past a lowered z1 are filtered when tested
        const uint64_t b1 = ballot(lL || rL), b2 = ballot(lL && rL);
        const int tot = __popcll(b1) + __popcll(b2);
        int pos = staged + __popcll(b1 & below) + __popcll(b2 & below);
        if (lL) M.c.st_id[pos++] = ~cl;
        if (rL) M.c.st_id[pos] = ~cr;
        staged += tot;
      }
    }
    const bool done = sp == 0;
    // tests of staged leaves, 64 at a time, in staging order: the bounding
    // sphere of the ellipsoid against the packet gives the entry's depth bounds
    while (staged >= 64 || (done && staged > 0)) {
      __builtin_amdgcn_wave_barrier();
      const int k = min(64, staged);
      if (count + k > kListCap) {
        // the list may overflow: pause at the smallest pending Z index if
        // the entries below it make a chunk
        int zq = sp > 0 ? M.c.ring_first[sp - 1] : z1;
        for (int e = lane; e < staged; e += 64) zq = min(zq, M.c.st_id[e]);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) zq = min(zq, __shfl_xor(zq, o, 64));
        zq = min(__builtin_amdgcn_readfirstlane(zq), z1);
        int nb = 0;
        for (int e0 = 0; e0 < count; e0 += 64)
          nb += __popcll(ballot(e0 + lane < count && M.l_id[e0 + lane] < zq));
        if (nb > 0) {
          t.sp = sp; t.staged = staged; t.count = count; t.visits = visits; t.z1 = z1;
          t.zp = zq;
          t.paused = true;
          nodes_out += visits - visits0;
          return sort_list(M, lane, count, zq);
        }
      }
      int j = 0;
      bool test = false;
      if (lane < k) {
        j = M.c.st_id[lane];
        test = j < z1;
      }
      bool keep = false;
      float tmin = 0.0f, tmax = 0.0f;
      if (test) {
        const vf4 *gp = reinterpret_cast<const vf4 *>(s.geom) + 4 * j;
        const vf4 g0 = gp[0], g3 = gp[3];
        // the support-function record is fetched with the geometry, before
        // the sphere test decides whether it is needed: one memory round
        // trip per batch of leaves instead of two
        vf4 x0 = {0.0f, 0.0f, 0.0f, 0.0f}, x1 = x0;
        if (cone.narrow) {
          const vf4 *ap = reinterpret_cast<const vf4 *>(s.aux) + 2 * j;
          x0 = ap[0];
          x1 = ap[1];
        }
        pin_loaded(g0); pin_loaded(g3); pin_loaded(x0); pin_loaded(x1);
        const float vx = g0.x - self.ox, vy = g0.y - self.oy, vz = g0.z - self.oz;
        keep = cone_sphere(cone, vx, vy, vz, g3.w, &tmin, &tmax);
        if (keep && cone.narrow) {
          float lo, hi;
          const bool in_cone = support_bounds(cone, vx, vy, vz, sqrtf(g0.w), x0.x, x0.y, x0.z,
                                              x0.w, x1.x, x1.y, x1.z, &lo, &hi);
          tmin = fmaxf(tmin, lo);
          tmax = fminf(tmax, hi);
          keep = in_cone && tmin <= cone.t_hi && tmax >= cone.t_lo;
        }
      }
      if (stats && ballot(test)) {
        const int64_t c0 = clock64();
        // statistics only: AABB-only leaves per ray (box met, ellipsoid missed)
        const Gauss g = with_origin(load_gauss_lane(s.geom, test ? j : 0), self.ox, self.oy, self.oz);
        const float *bx = s.aabb + 6 * (size_t)(test ? j : 0);
        for (uint64_t rem = rays; rem; rem &= rem - 1) {
          const int r = __builtin_ctzll(rem);
          const Ray q = lds_ray(M, self, r);
          const float lo = M.rlo[r], hi = M.rhi[r];
          if (!test || !box_hit(bx[0], bx[1], bx[2], bx[3], bx[4], bx[5], q, lo, hi)) continue;
          const Chord ch = chord(g, q);
          if (!(ch.exists && ch.tin <= hi && ch.tout >= lo)) atomicAdd(&M.cnt_box[r], 1);
        }
        if (cyc_excl) *cyc_excl += clock64() - c0;
      }
      leaves_out += k;
      int tot = __popcll(ballot(keep));
      if (count + tot > kListCap) {
        // list overflow: lower z1 so that half the list remains
        int v[kListCap / 64 + 1];
        bool ok[kListCap / 64 + 1];
#pragma unroll
        for (int q = 0; q < kListCap / 64; q++) {
          const int e = lane + 64 * q;
          ok[q] = e < count;
          v[q] = ok[q] ? M.l_id[e] : 0;
        }
        v[kListCap / 64] = j;
        ok[kListCap / 64] = keep;
        z1 = select_cut(v, ok, z0 + 1, z1, kListCap / 2);
        count = compact_list(M, lane, count, z1);
        keep = keep && j < z1;
        tot = __popcll(ballot(keep));
      }
      const uint64_t bk = ballot(keep);
      if (keep) {
        const int pos = count + __popcll(bk & below);
        M.l_id[pos] = j;
        M.l_tin[pos] = tmin;
        M.l_tout[pos] = tmax;
      }
      count += tot;
      // move the remaining staged entries to the front
      const int rest = staged - k;
      int rid[2];
      for (int e = 0; e < 2; e++) {
        const int src = k + lane + 64 * e;
        if (lane + 64 * e < rest) rid[e] = M.c.st_id[src];
      }
      __builtin_amdgcn_wave_barrier();
      for (int e = 0; e < 2; e++) {
        const int dst = lane + 64 * e;
        if (dst < rest) M.c.st_id[dst] = rid[e];
      }
      staged = rest;
    }
    if (done && staged == 0) break;
  }
  nodes_out += visits - visits0;
  t.sp = 0; t.staged = 0; t.count = count; t.visits = visits; t.z1 = z1;
  t.zp = z1;
  t.paused = false;
  return sort_list(M, lane, count, z1);
}

// ---------------------------------------------------------------------------
// Sources of a segment's candidate Gaussians, both in Z-index order: the
// window list (LDS) or every active Gaussian (brute force).

enum SourceKind { SRC_LIST = 0, SRC_BRUTE = 1 };

// Reads lane `src`'s copy of a geometry record (wave-uniform result).
__device__ __forceinline__ Gauss gauss_from_lane(const Gauss &v, int src) {
  Gauss g;
  auto rl = [src](float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), src));
  };
  g.mx = rl(v.mx); g.my = rl(v.my); g.mz = rl(v.mz); g.k2 = rl(v.k2);
#pragma unroll
  for (int k = 0; k < 9; k++) g.m[k] = rl(v.m[k]);
  g.sig = rl(v.sig); g.l2sig = rl(v.l2sig); g.rad = rl(v.rad);
  g.ox = rl(v.ox); g.oy = rl(v.oy); g.oz = rl(v.oz);
  return g;
}

// Entries of M.order carry a mark bit above the slot index: set by a MARK
// pass for the entries some lane hit, read by a FILTER pass over the same
// list and the same segments.
constexpr int kOrderMark = 1 << 16;
enum CandMode { CAND_ALL = 0, CAND_MARK = 1, CAND_FILTER = 2 };

// Calls fn(j, g) for every candidate j with its geometry record g.
// `a_min`/`b_max` bound the live lanes' segments for the list's uniform
// depth pre-check.  List entries are taken 64 at a time: lane i holds entry
// base + i and loads that entry's geometry, so one memory round trip serves
// the whole block; the surviving candidates are then read back with readlane.
// CAND_MARK: fn returns whether some lane hit the candidate, and the entry's
// mark is set to that; CAND_FILTER: only marked entries are visited (list
// source only; the brute-force source visits everything).
// With use_marks, a CAND_MARK pass trusts the marks already set (from a
// record of the same pass) and visits only the marked entries.
template <int MODE = CAND_ALL, class Fn>
__device__ __forceinline__ void for_each_candidate(int kind, const SceneDev &s, WaveMem &M,
                                                   int count, int lane, float a_min, float b_max,
                                                   int n_active, const Ray &r, Fn &&fn,
                                                   bool use_marks = false) {
  const float ox = r.ox, oy = r.oy, oz = r.oz;
  if (kind == SRC_LIST) {
    for (int base = 0; base < count; base += 64) {
      const int e = base + lane;
      int id = 0, o = 0;
      bool keep = false;
      if (e < count) {
        const int om = M.order[e];
        o = om & (kOrderMark - 1);
        // the entry's three words are read together (no short-circuit
        // between the depth tests, which would wait for each read in turn)
        const float tin = M.l_tin[o], tout = M.l_tout[o];
        id = M.l_id[o];
        keep = !(tin > b_max) & !(tout < a_min);
        if (MODE == CAND_FILTER || (MODE == CAND_MARK && use_marks))
          keep = keep & ((om & kOrderMark) != 0);
      }
      const uint64_t bits0 = ballot(keep);
      if (!bits0) continue;
      const Gauss mine = with_origin(load_gauss_lane(s.geom, keep ? id : 0), ox, oy, oz);
      uint64_t hits = 0;   // (uniform) the block's candidates some lane hit
      for (uint64_t bits = bits0; bits; bits &= bits - 1) {
        const int src = __builtin_ctzll(bits);
        if constexpr (MODE == CAND_MARK) {
          if (fn(__builtin_amdgcn_readlane(id, src), gauss_from_lane(mine, src))) hits |= 1ull << src;
        } else {
          fn(__builtin_amdgcn_readlane(id, src), gauss_from_lane(mine, src));
        }
      }
      if (MODE == CAND_MARK && !use_marks && keep)
        M.order[e] = o | (((hits >> lane) & 1ull) ? kOrderMark : 0);
    }
  } else {
    for (int e = 0; e < n_active; e++) fn(e, with_origin(load_gauss(s.geom, e), ox, oy, oz));
  }
}

// Window-list record of a tile (layout next to kWrecHeader): a forward
// appends every collection's sorted chunk with the collection state its
// callers read, and after every pass over a list the marks of the entries
// some lane hit; a backward of the same rays reads them back in the same
// order instead of walking the tree, and visits only the marked entries.
// Every record starts with the offset of the tile's next record.
struct WinRec {
  uint32_t *slot = nullptr;   // the tile's (complete, first record) pair
  uint32_t cur = kWrecNone;   // replay: next record to read; record: last record written
  uint32_t first = kWrecNone; // record: first record
  bool ok = false;            // record: nothing dropped so far; replay: tile complete
};

__device__ __forceinline__ void rec_start(WinRec &R, const MarchOpts &op, const ViewTable &vt,
                                          int w) {
  R.slot = op.replay_mode ? op.wrec_tile + 2 * (size_t)(vt.tile0 + w) : nullptr;
  R.cur = kWrecNone;
  R.first = kWrecNone;
  R.ok = false;
  if (op.replay_mode == 1) {
    R.ok = true;
  } else if (op.replay_mode == 2) {
    R.ok = uniform_int((int)R.slot[0]) == 1;
    R.cur = (uint32_t)uniform_int((int)R.slot[1]);
  }
}

// forward: the tile's status once all its records are in
__device__ __forceinline__ void rec_finish(WinRec &R, const MarchOpts &op, int lane) {
  if (op.replay_mode != 1) return;
  if (lane == 0) {
    R.slot[0] = R.ok ? 1u : 0u;
    R.slot[1] = R.first;
  }
}

// Appends a record of `size` dwords to the tile's chain; kWrecNone (and the
// tile marked incomplete) when the pool is full.
__device__ __forceinline__ uint32_t rec_alloc(WinRec &R, const MarchOpts &op, uint32_t size,
                                              int lane) {
  // a 64-bit allocation counter (pool dwords 0-1): failed allocations keep
  // adding to it, and it must not wrap back into the pool
  unsigned long long got = 0;
  if (lane == 0) got = atomicAdd(reinterpret_cast<unsigned long long *>(op.wrec), (unsigned long long)size);
  const uint64_t at = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(got >> 32)) << 32) |
                      (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)got);
  if (at + size > op.wrec_cap) { R.ok = false; return kWrecNone; }
  const uint32_t off = (uint32_t)at;
  if (lane == 0) {
    op.wrec[off] = kWrecNone;
    if (R.cur != kWrecNone) op.wrec[R.cur] = off;   // link from the previous record
  }
  if (R.first == kWrecNone) R.first = off;
  R.cur = off;
  return off;
}

// Checks that a record of at least `size` dwords at `off` lies in the pool.
__device__ __forceinline__ bool rec_fits(const MarchOpts &op, uint32_t off, uint64_t size) {
  return off < op.wrec_cap && (uint64_t)off + size <= op.wrec_cap;
}

__device__ __forceinline__ void rec_put(WinRec &R, const MarchOpts &op, const WaveMem &M,
                                        const Trav &t, int cnt, int lane) {
  if (!R.ok) return;
  const int n = cnt > 0 ? cnt : 0;
  const uint32_t off = rec_alloc(R, op, kWrecHeader + 3 * n, lane);
  if (off == kWrecNone) return;
  uint32_t *p = op.wrec + off;
  if (lane == 0) {
    p[1] = (uint32_t)cnt; p[2] = t.paused ? 1u : 0u; p[3] = (uint32_t)t.z0;
    p[4] = (uint32_t)t.z1; p[5] = (uint32_t)t.zp; p[6] = (uint32_t)t.count;
  }
  for (int e = lane; e < n; e += 64) {
    const int o = M.order[e] & (kOrderMark - 1);
    p[kWrecHeader + 3 * e] = (uint32_t)M.l_id[o];
    p[kWrecHeader + 3 * e + 1] = __float_as_uint(M.l_tin[o]);
    p[kWrecHeader + 3 * e + 2] = __float_as_uint(M.l_tout[o]);
  }
}

// The marks of the current list's `count` entries after a pass: [next, count,
// then one 64-bit ballot per 64 entries].
__device__ __forceinline__ void rec_put_marks(WinRec &R, const MarchOpts &op, const WaveMem &M,
                                              int count, int lane) {
  if (!R.ok) return;
  const int words = (count + 63) >> 6;
  const uint32_t off = rec_alloc(R, op, 2 + 2 * words, lane);
  if (off == kWrecNone) return;
  uint32_t *p = op.wrec + off;
  if (lane == 0) p[1] = (uint32_t)count;
  for (int q = 0; q < words; q++) {
    const int e = 64 * q + lane;
    const uint64_t b = ballot(e < count && (M.order[e] & kOrderMark) != 0);
    if (lane == 0) {
      p[2 + 2 * q] = (uint32_t)b;
      p[3 + 2 * q] = (uint32_t)(b >> 32);
    }
  }
}

// The per-sample sums of a segment step (layout next to kSrecHeader): lanes
// `hit` store sigma_k and W_k, lanes `empty` their restart distance.
template <int NS>
__device__ __forceinline__ void rec_put_samples(WinRec &R, const MarchOpts &op, bool hit,
                                                bool empty, float best, const float *sg,
                                                const float *W0, const float *W1,
                                                const float *W2, int lane) {
  if (!R.ok) return;
  const uint64_t hm = ballot(hit), em = ballot(empty);
  const int nh = __popcll(hm), ne = __popcll(em);
  const uint32_t off = rec_alloc(R, op, kSrecHeader + 4 * NS * nh + ne, lane);
  if (off == kWrecNone) return;
  uint32_t *p = op.wrec + off;
  if (lane == 0) {
    p[1] = (uint32_t)hm; p[2] = (uint32_t)(hm >> 32);
    p[3] = (uint32_t)em; p[4] = (uint32_t)(em >> 32);
  }
  float *q = reinterpret_cast<float *>(p + kSrecHeader);
  const uint64_t below = lanes_below(lane);
  if (hit) {
    const int rk = __popcll(hm & below);
#pragma unroll
    for (int k = 0; k < NS; k++) {
      q[(4 * k) * nh + rk] = sg[k];
      q[(4 * k + 1) * nh + rk] = W0[k];
      q[(4 * k + 2) * nh + rk] = W1[k];
      q[(4 * k + 3) * nh + rk] = W2[k];
    }
  }
  if (empty) q[4 * NS * nh + __popcll(em & below)] = best;
}

// Reads the sample record of a segment step back: sigma_k into sg, G . W_k
// into GW, and for an empty segment the restart distance into *best.
// Returns whether this lane's segment hit something.  A record that does not
// match the lanes that march (cannot happen) is reported, and its lanes read
// as empty with no restart.
template <int NS>
__device__ __forceinline__ bool rec_get_samples(WinRec &R, const MarchOpts &op, bool go, float Gc0,
                                                float Gc1, float Gc2, float *sg, float *GW,
                                                float *best, int lane, int32_t *err) {
  *best = kInf;
  const uint32_t off = R.cur;
  if (off == kWrecNone || !rec_fits(op, off, kSrecHeader)) {
    if (err) *err = 5;
    R.cur = kWrecNone;
    return false;
  }
  const uint32_t *p = op.wrec + off;
  // the header's five words in one batch of loads
  uint32_t hw[kSrecHeader];
#pragma unroll
  for (int i = 0; i < kSrecHeader; i++) hw[i] = p[i];
#pragma unroll
  for (int i = 0; i < kSrecHeader; i++) pin_lane(hw[i]);
  const uint64_t hm = ((uint64_t)(uint32_t)uniform_int((int)hw[2]) << 32) | (uint32_t)uniform_int((int)hw[1]);
  const uint64_t em = ((uint64_t)(uint32_t)uniform_int((int)hw[4]) << 32) | (uint32_t)uniform_int((int)hw[3]);
  const int nh = __popcll(hm), ne = __popcll(em);
  if ((hm | em) != ballot(go) || (hm & em) != 0 ||
      !rec_fits(op, off, kSrecHeader + 4 * (uint64_t)NS * nh + ne)) {
    if (err) *err = 5;
    R.cur = kWrecNone;
    return false;
  }
  R.cur = (uint32_t)uniform_int((int)hw[0]);
  const float *q = reinterpret_cast<const float *>(p + kSrecHeader);
  const uint64_t below = lanes_below(lane);
  const bool hit = (hm >> lane) & 1ull;
  if (hit) {
    const int rk = __popcll(hm & below);
    // the 4 N_s values in one batch of loads (the compiler would otherwise
    // wait for every few of them in turn to keep fewer registers live)
    float v[4 * NS];
#pragma unroll
    for (int i = 0; i < 4 * NS; i++) v[i] = q[i * nh + rk];
#pragma unroll
    for (int i = 0; i < 4 * NS; i++) pin_lane(__float_as_uint(v[i]));
#pragma unroll
    for (int k = 0; k < NS; k++) {
      sg[k] = v[4 * k];
      GW[k] = fmaf(Gc0, v[4 * k + 1], fmaf(Gc1, v[4 * k + 2], Gc2 * v[4 * k + 3]));
    }
  }
  if ((em >> lane) & 1ull) *best = q[4 * NS * nh + __popcll(em & below)];
  return hit;
}

// Loads the chunk at pool offset `off` into the list (identity order, no
// marks); returns its collection's result and the next record in *next.
__device__ __forceinline__ int rec_load(const MarchOpts &op, WaveMem &M, uint32_t off, int lane,
                                        uint32_t *next) {
  // a record always fits the pool and the list; anything else is reported
  if (!rec_fits(op, off, kWrecHeader)) { *next = kWrecNone; return -1; }
  const uint32_t *p = op.wrec + off;
  const int cnt = uniform_int((int)p[1]);
  const int n = cnt > 0 ? cnt : 0;
  if (n > kListCap || !rec_fits(op, off, kWrecHeader + 3 * (uint64_t)n)) {
    *next = kWrecNone;
    return -1;
  }
  __builtin_amdgcn_wave_barrier();
  for (int e = lane; e < n; e += 64) {
    M.l_id[e] = (int)p[kWrecHeader + 3 * e];
    M.l_tin[e] = __uint_as_float(p[kWrecHeader + 3 * e + 1]);
    M.l_tout[e] = __uint_as_float(p[kWrecHeader + 3 * e + 2]);
    M.order[e] = e;
  }
  __builtin_amdgcn_wave_barrier();
  *next = (uint32_t)uniform_int((int)p[0]);
  return cnt;
}

// Sets the list's marks from the marks record at `off` (which must cover
// `count` entries); false on a broken record.
__device__ __forceinline__ bool rec_load_marks(const MarchOpts &op, WaveMem &M, uint32_t off,
                                               int count, int lane, uint32_t *next) {
  const int words = (count + 63) >> 6;
  if (!rec_fits(op, off, 2 + 2 * (uint64_t)words)) { *next = kWrecNone; return false; }
  const uint32_t *p = op.wrec + off;
  const uint32_t h0 = p[0], h1 = p[1];
  pin_lane(h0); pin_lane(h1);
  constexpr int kSlots = kListCap / 64;
  if (uniform_int((int)h1) != count || words > kSlots) { *next = kWrecNone; return false; }
  __builtin_amdgcn_wave_barrier();
  if (words > 0) {
    // every mark word in one batch of loads (slots past the end read the
    // last word again and are not used)
    uint32_t w[kSlots];
#pragma unroll
    for (int q = 0; q < kSlots; q++) w[q] = p[2 + 2 * min(q, words - 1) + (lane >> 5)];
#pragma unroll
    for (int q = 0; q < kSlots; q++) pin_lane(w[q]);
#pragma unroll
    for (int q = 0; q < kSlots; q++) {
      const int e = 64 * q + lane;
      if (q < words && e < count) {
        const int o = M.order[e] & (kOrderMark - 1);
        M.order[e] = o | (((w[q] >> (lane & 31)) & 1u) ? kOrderMark : 0);
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
  *next = (uint32_t)uniform_int((int)h0);
  return true;
}

// Backward pass over the current list: in a replayed tile, the forward's
// marks of this pass (true: visit only those), else false (mark as it goes).
__device__ __forceinline__ bool rec_next_marks(WinRec &R, const MarchOpts &op, WaveMem &M,
                                               int count, int kind, int lane, int32_t *err) {
  if (!(op.replay_mode == 2 && R.ok) || kind != SRC_LIST) return false;
  uint32_t next;
  if (R.cur == kWrecNone || !rec_load_marks(op, M, R.cur, count, lane, &next)) {
    // a broken record (cannot happen): flag it; later reads of this tile's
    // record find no next record and end its rays
    if (err) *err = 5;
    R.cur = kWrecNone;
    return false;
  }
  R.cur = next;
  return true;
}

// One collection: the tree walk (recorded in a recording forward) or, in a
// replaying backward of a complete tile, the recorded chunk and state.
// *start receives the chunk's record offset.
// REPLAY false (the forward kernel) compiles the replay branch out: a
// forward never reads a record, and the branch's registers would count
// against the whole kernel.
template <bool REPLAY>
__device__ __forceinline__ int collect(const SceneDev &s, const MarchOpts &op, WaveMem &M,
                                       const Ray &r, int lane, Trav &t, int n_active, bool stats,
                                       int32_t *err, int32_t &nodes, int32_t &leaves,
                                       int64_t *cyc_excl, WinRec &R, uint32_t *start) {
  if (REPLAY && op.replay_mode == 2 && R.ok) {
    if (R.cur == kWrecNone || !rec_fits(op, R.cur, kWrecHeader)) {   // a broken record
      if (err) *err = 5;
      t.count = 0;
      t.paused = false;
      return -1;
    }
    const uint32_t *p = op.wrec + R.cur;
    t.paused = uniform_int((int)p[2]) != 0;
    t.z0 = uniform_int((int)p[3]);
    t.z1 = uniform_int((int)p[4]);
    t.zp = uniform_int((int)p[5]);
    t.count = uniform_int((int)p[6]);
    *start = R.cur;
    uint32_t next;
    const int cnt = rec_load(op, M, R.cur, lane, &next);
    if (cnt < 0 && err) *err = 5;
    R.cur = next;
    return cnt;
  }
  // the walk is a chain of dependent loads and short bursts of work: while
  // it runs, the wave's instructions issue ahead of other waves' long
  // arithmetic runs on the same SIMD (wave priority, not a queue priority)
  __builtin_amdgcn_s_setprio(3);
  const int cnt = trav_run(s, M, r, lane, t, n_active, stats, err, nodes, leaves, cyc_excl);
  __builtin_amdgcn_s_setprio(0);
  if (op.replay_mode == 1) rec_put(R, op, M, t, cnt, lane);
  *start = R.cur;
  return cnt;
}

// Per-wave window bookkeeping shared by forward and backward.
struct Window {
  float len, len_min, len_max;   // uniform window length beyond the segment, and its bounds
  bool valid;                    // per lane: the current list covers this lane's later segments
  float hi;                      // per lane window end
  int count;                     // uniform number of candidates in M.order
  int kind;                      // SourceKind of the current candidates
  bool chunked;                  // uniform: this segment's candidates come in Z chunks
  int zend;                      // uniform end of the Z range the chunks cover
  uint32_t rec_first, rec_last;  // record offsets of the segment's first and last chunk
  Trav t;                        // the collection behind the list
};

// Makes sure every live lane whose segment fits its window can march; when
// no live lane can, collects a new window for all live lanes.  A window that
// could not be collected whole serves the current segment only, chunk by
// chunk.
template <bool REPLAY>
__device__ __forceinline__ void ensure_window(const SceneDev &s, const MarchOpts &op, WaveMem &M,
                                              const Ray &r, int lane, int n_active, bool alive,
                                              float a, float b, Window &w, bool stats,
                                              int32_t *err, int32_t &nodes, int32_t &leaves,
                                              int32_t &windows, bool &fits, WinRec &R,
                                              int64_t *cyc_excl = nullptr) {
  if (op.brute_force) {
    w.kind = SRC_BRUTE;
    w.chunked = false;
    fits = alive;
    return;
  }
  fits = alive && w.valid && b <= w.hi;
  if (ballot(fits) != 0 || ballot(alive) == 0) {
    w.chunked = false;
    return;
  }
  const uint64_t rays = ballot(alive);
  const float hi = alive ? fmaxf(a + w.len, b) : -kInf;
  M.rlo[lane] = alive ? a : kInf;
  M.rhi[lane] = hi;
  windows++;
  trav_start(M, lane, w.t, rays, 0, n_active);
  w.zend = n_active;
  const int cnt = collect<REPLAY>(s, op, M, r, lane, w.t, n_active, stats, err, nodes, leaves,
                                  cyc_excl, R, &w.rec_first);
  w.rec_last = w.rec_first;
  w.kind = SRC_LIST;
  w.count = cnt > 0 ? cnt : 0;   // a malformed tree ends the rays (error flag set)
  w.chunked = cnt >= 0 && (w.t.paused || w.t.z1 < n_active);
  if (!w.chunked) {
    w.valid = alive;
    w.hi = hi;
    if (w.t.count < kListCap / 4) w.len = fminf(fmaxf(w.len * 1.5f, w.len_min), w.len_max);
  } else {
    w.valid = false;
    w.len = w.len * 0.5f < w.len_min ? 0.0f : w.len * 0.5f;
  }
  fits = alive;
}

// Starts the chunks of the current segment again over the Z range [0, zend),
// for the lanes in `lanes` over their segments [a, b].
__device__ __forceinline__ void first_chunk(const SceneDev &s, WaveMem &M, const Ray &r, int lane,
                                            int n_active, bool lanes, float a, float b, int zend,
                                            Window &w, bool stats, int32_t *err, int32_t &nodes,
                                            int32_t &leaves, int32_t &windows) {
  const uint64_t rays = ballot(lanes);
  M.rlo[lane] = lanes ? a : kInf;
  M.rhi[lane] = lanes ? b : -kInf;
  windows++;
  trav_start(M, lane, w.t, rays, 0, zend);
  w.zend = zend;
  const int cnt = trav_run(s, M, r, lane, w.t, n_active, stats, err, nodes, leaves, nullptr);
  w.count = cnt > 0 ? cnt : 0;
}

// In chunked mode, moves to the candidates of the next Z chunk: resumes a
// paused collection, or after a cut at z1 collects again from z1 for the
// lanes in `lanes` over their segments [a, b].  False when the segment's
// candidates are exhausted.
template <bool REPLAY>
__device__ __forceinline__ bool next_chunk(const SceneDev &s, const MarchOpts &op, WaveMem &M,
                                           const Ray &r, int lane, int n_active, bool lanes,
                                           float a, float b, Window &w, bool stats, int32_t *err,
                                           int32_t &nodes, int32_t &leaves, int32_t &windows,
                                           WinRec &R, int64_t *cyc_excl = nullptr) {
  if (!w.chunked) return false;
  if (w.t.paused) {
    if (!(REPLAY && op.replay_mode == 2 && R.ok)) trav_advance(M, lane, w.t);
  } else {
    if (w.t.z1 >= w.zend) return false;
    const uint64_t rays = ballot(lanes);
    if (rays == 0) return false;
    M.rlo[lane] = lanes ? a : kInf;
    M.rhi[lane] = lanes ? b : -kInf;
    windows++;
    trav_start(M, lane, w.t, rays, w.t.z1, w.zend);
  }
  const int cnt = collect<REPLAY>(s, op, M, r, lane, w.t, n_active, stats, err, nodes, leaves,
                                  cyc_excl, R, &w.rec_last);
  if (cnt < 0) {
    w.count = 0;
    w.chunked = false;
    return false;
  }
  w.count = cnt;
  return true;
}

// ---------------------------------------------------------------------------
// Forward kernel (and the hit-dump variant).

template <int NS, bool DUMP, bool STATS, bool SG = false>
__global__ __launch_bounds__(kWave, NS <= 8 ? 3 : 2) void k_forward(SceneDev s, ViewTable vt, MarchOpts op,
                                                   FwdOut out, LaunchShape ls) {
  __shared__ WaveMem M;
  const int lane = threadIdx.x;
  const int n_active = uniform_int(s.counters[0]);
  const bool grid = !op.adaptive && op.ess != 2;
  constexpr bool stats = STATS;
  bool first = true;
  for (;;) {
    int w;
    if (op.persistent) {
      w = pop_tile(ls.queue, vt.n_tiles, blockIdx.x & 7, lane);
      if (w < 0) break;
    } else {
      if (!first) break;
      w = xcd_block(blockIdx.x, gridDim.x);
      if (w >= vt.n_tiles) break;
    }
    first = false;

    Pixel px;
    int dump_slot = 0;
    if (DUMP) {
      dump_slot = w * 64 + lane;
      px.view = 0;
      px.valid = dump_slot < out.dump_n;
      const int pix = px.valid ? out.dump_pix[dump_slot] : 0;
      px.px = pix % vt.v[0].width;
      px.py = pix / vt.v[0].width;
      px.ray = dump_slot;
    } else {
      px = tile_pixel(vt, op, w, lane);
    }
    const View &V = vt.v[px.view];
    const Ray r = make_ray(V, px.px, px.py);
    M.rdx[lane] = r.dx; M.rdy[lane] = r.dy; M.rdz[lane] = r.dz;
    M.rix[lane] = r.ix; M.riy[lane] = r.iy; M.riz[lane] = r.iz;
    M.cnt_box[lane] = 0;
    const float tn = V.t_near, tf = V.t_far;
    float Y[16];
    sh_basis(op.sh_k, r.dx, r.dy, r.dz, Y);

    SegState ss;
    int n_closest = 0;   // closest-hit queries of this lane's ray so far
    WinRec rec;
    rec_start(rec, op, vt, w);
    ss.alive = px.valid;
    ss.pending = op.ess && px.valid;
    ss.seg_i = 0;
    ss.a = tn;
    ss.cl_lo = tn;
    const float dS = op.dt * (float)NS;
    Window win;
    const float seg_max = (float)NS * (op.adaptive ? op.dt_max : op.dt);
    win.len_min = (float)NS * (op.adaptive ? op.dt_min : op.dt);
    win.len = (float)op.window_segments * seg_max;
    win.len_max = fmaxf(8.0f * seg_max, 2.0f * win.len);
    win.valid = false;
    win.hi = -kInf;
    win.count = 0;
    win.kind = SRC_LIST;
    win.chunked = false;
    win.t.paused = false;
    win.t.z1 = n_active;
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    int32_t cnt[kNStatUsed];
#pragma unroll
    for (int k = 0; k < kNStatUsed; k++) cnt[k] = 0;
    cnt[ST_T_END] = __float_as_int(tf);
    // statistics builds also time the phases of the tile (shader clock)
    int64_t cyc_collect = 0, cyc_closest = 0, cyc_t0 = 0, cyc_tile = stats ? clock64() : 0;
    int64_t cyc_boxstat = 0;   // statistics-only work inside the collection
    float prev_a = -kInf, prev_b = -kInf;
    int n_dump = 0;

    for (;;) {
      if (stats) cyc_t0 = clock64();
      if (op.ess)
        closest_pass(s, op, n_active, r, tn, tf, dS, ss, ls.error_flag,
                     stats ? &cnt[ST_CLOSEST] : nullptr, n_closest, px.ray);
      if (stats) cyc_closest += clock64() - cyc_t0;
      if (ss.alive) {
        const float a0 = grid ? fmaf((float)(ss.seg_i * NS), op.dt, tn) : ss.a;
        if (!(a0 < tf)) ss.alive = false;
        else if (!(T > op.t_eps)) {
          ss.alive = false;
          if (stats) cnt[ST_T_END] = __float_as_int(a0);
        }
      }
      if (ballot(ss.alive) == 0) break;
      float a = 0.0f, b = 0.0f, dt = op.dt;
      Samples sp;
      if (ss.alive) {
        if (!segment<NS>(op, grid, ss, tn, T, a, b, dt, sp)) {   // no progress in FP32
          ss.alive = false;
          if (ls.error_flag) *ls.error_flag = 4;
        }
      }
      if (!ss.alive) { sp.t0 = 0.0f; sp.dt = 0.0f; }
      bool go;
      if (stats) cyc_t0 = clock64();
      ensure_window<false>(s, op, M, r, lane, n_active, ss.alive, a, b, win, stats, ls.error_flag,
                    cnt[ST_NODES], cnt[ST_LEAVES], cnt[ST_WINDOWS], go, rec,
                    stats ? &cyc_boxstat : nullptr);
      if (stats) cyc_collect += clock64() - cyc_t0;
      if (stats && go && win.chunked) cnt[ST_CHUNKED]++;
      const float a_min = wave_min(go ? a : kInf), b_max = wave_max(go ? b : -kInf);
      const float lo = go ? a : kInf, hi = go ? b : -kInf;
      float sg[NS], W0[NS], W1[NS], W2[NS];
#pragma unroll
      for (int k = 0; k < NS; k++) { sg[k] = 0.0f; W0[k] = W1[k] = W2[k] = 0.0f; }
      int nhit = 0;

      do {
        for_each_candidate<CAND_MARK>(win.kind, s, M, win.count, lane, a_min, b_max, n_active, r,
                                      [&](int j, const Gauss &g) {
        const bool want = go;
        if (stats) cnt[ST_CAND]++;
        const Chord c = chord(g, r);
        // one conjunction, not a chain of short-circuit branches: the test
        // stays in lane masks, with no branch per term
        const bool hit = want & c.exists & (c.tin <= hi) & (c.tout >= lo);
        if (ballot(hit) == 0) return false;
        if (stats) cnt[ST_CAND_HIT]++;
        if (hit) {
          nhit++;
          if (stats && !(c.tin <= prev_b && c.tout >= prev_a)) cnt[ST_Q]++;
          if (DUMP) {
            if (n_dump < out.dump_cap) {
              out.dump_a[(size_t)dump_slot * out.dump_cap + n_dump] = a;
              out.dump_ids[(size_t)dump_slot * out.dump_cap + n_dump] = (int32_t)s.perm[j];
            }
            n_dump++;
          }
          // the colour record's loads go out before the sample weights,
          // which do not need them
          const ColRec rc = colour_load(s.col, j);
          float wk[NS];
          const uint32_t live = sample_weights<NS, true>(g, c, sp, wk);
          float cr, cg, cb;
          colour_eval(rc, Y, cr, cg, cb);
          if constexpr (SG) sg_colour(s.sg, j, r.dx, r.dy, r.dz, cr, cg, cb);
#pragma unroll
          for (int k = 0; k < NS; k++) {
            if (!(live & (1u << k))) continue;
            sg[k] += wk[k];
            W0[k] = fmaf(wk[k], cr, W0[k]);
            W1[k] = fmaf(wk[k], cg, W1[k]);
            W2[k] = fmaf(wk[k], cb, W2[k]);
          }
        }
        return true;
      });
        // the entries this pass hit, for a replaying backward
        if (op.replay_mode == 1 && win.kind == SRC_LIST) rec_put_marks(rec, op, M, win.count, lane);
      } while ([&] {
        if (stats) cyc_t0 = clock64();
        const bool more = next_chunk<false>(s, op, M, r, lane, n_active, go, a, b, win, stats,
                                     ls.error_flag, cnt[ST_NODES], cnt[ST_LEAVES], cnt[ST_WINDOWS],
                                     rec, stats ? &cyc_boxstat : nullptr);
        if (stats) cyc_collect += clock64() - cyc_t0;
        return more;
      }());

      // an empty segment restarts at the next closest hit: inside the window
      // from the list, otherwise through a closest-hit traversal
      const bool empty = go && nhit == 0;
      float best = kInf;
      if (op.ess && win.kind == SRC_LIST && !win.chunked && ballot(empty)) {
        const float bmin = wave_min(empty ? b : kInf);
        for_each_candidate(SRC_LIST, s, M, win.count, lane, bmin, kInf, n_active, r,
                           [&](int j, const Gauss &g) {
          const bool want = empty;
          const Chord c = chord(g, r);
          if (want && c.exists && c.tout >= b && c.tin <= win.hi) best = fminf(best, fmaxf(c.tin, b));
        });
      }
      // the step's per-sample sums and restarts, for a replaying backward
      if (op.replay_mode == 1 && op.sample_rec)
        rec_put_samples<NS>(rec, op, go && nhit > 0, empty, best, sg, W0, W1, W2, lane);
      if (go) {
        if (nhit > 0) {
          if (stats) { cnt[ST_SEGMENTS]++; cnt[ST_P] += nhit; }
#pragma unroll
          for (int k = 0; k < NS; k++) {
            if (sp.t(k) < tf) {
              if (stats) cnt[ST_SAMPLES]++;
              if (sg[k] > 0.0f) {
                const float x = sg[k] * dt;
                const float f = T * (one_minus_exp_neg(x) * __builtin_amdgcn_rcpf(sg[k]));
                C0 = fmaf(f, W0[k], C0);
                C1 = fmaf(f, W1[k], C1);
                C2 = fmaf(f, W2[k], C2);
                T *= exp_neg(x);
              }
            }
          }
          prev_a = a;
          prev_b = b;
        }
        step_after(op, grid, nhit > 0, best, tn, dS, b, ss);
      }
    }

    rec_finish(rec, op, lane);
    if (stats) {
      cnt[ST_BOX_ONLY] += M.cnt_box[lane];
      cnt[ST_KCYC_COLLECT] = (int32_t)((cyc_collect - cyc_boxstat) >> 10);
      cnt[ST_KCYC_CLOSEST] = (int32_t)(cyc_closest >> 10);
      cnt[ST_KCYC_TILE] = (int32_t)((clock64() - cyc_tile - cyc_boxstat) >> 10);
    }
    if (DUMP) {
      if (px.valid) out.dump_count[dump_slot] = n_dump;
    } else if (px.valid) {
      out.rgb[3 * (size_t)px.ray + 0] = fmaf(T, op.bg[0], C0);
      out.rgb[3 * (size_t)px.ray + 1] = fmaf(T, op.bg[1], C1);
      out.rgb[3 * (size_t)px.ray + 2] = fmaf(T, op.bg[2], C2);
      out.T[px.ray] = T;
      if (stats) {
        for (int k = 0; k < kNStatUsed; k++) out.stats[(size_t)px.ray * kNStat + k] = cnt[k];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Lobe gradients of Gaussian j for one pass-B visit.  The lane's dL/dc is
// S G (S = sum_k w_k T_k phi_k, zero where the lane missed j), so per lobe
// with g = exp(lambda (u.d - 1)) and A = a.G:
//   dL/da = S g G,  dL/dlambda = S A g (u.d - 1),  h = S A g d,
// h being dL/du / lambda (the finalisation multiplies by lambda and takes
// the component across u).  Two lobes (16 slots) at a time are summed over
// the wave and added with one atomic per slot.
__device__ __forceinline__ void sg_slots(const float *sg, float *sgacc, int j, float S, float G0,
                                         float G1, float G2, const Ray &r, int lane) {
  cfloat4p p = as_const4(sg) + (size_t)(kSgFloats / 4) * j;
#pragma unroll 1
  for (int pair = 0; pair < (kMaxSg + 1) / 2; pair++) {
    float v[16];
#pragma unroll
    for (int h = 0; h < 2; h++) {
      const int k = 2 * pair + h;
      float *o = v + 8 * h;
      if (k < kMaxSg) {
        const vf4 a = p[2 * k], u = p[2 * k + 1];
        const float cosang = fmaf(u.x, r.dx, fmaf(u.y, r.dy, u.z * r.dz));
        const float sgv = S * __builtin_amdgcn_exp2f(a.w * kLog2e * (cosang - 1.0f));
        const float sa = sgv * fmaf(a.x, G0, fmaf(a.y, G1, a.z * G2));
        o[0] = sgv * G0; o[1] = sgv * G1; o[2] = sgv * G2;
        o[3] = sa * (cosang - 1.0f);
        o[4] = sa * r.dx; o[5] = sa * r.dy; o[6] = sa * r.dz;
        o[7] = 0.0f;
      } else {
#pragma unroll
        for (int e = 0; e < 8; e++) o[e] = 0.0f;
      }
    }
    const float mine = wave_sum_slots16(v, lane);
    if ((lane & 3) == 0 && 16 * pair + (lane >> 2) < kMaxSg * kSgLobeFloats)
      unsafeAtomicAdd(sgacc + (size_t)kSgAccFloats * j + 16 * pair + (lane >> 2), mine);
  }
}

// ---------------------------------------------------------------------------
// Backward kernel: replays the forward's segments from the same window lists
// (or brute force / depth-first sources) in the same order, takes each
// segment's per-sample sums from the forward's record (or sums them again
// where there is none), recomputes the transmittance before every sample,
// derives dL/dsigma_k and dL/dW_k, then revisits the Gaussians some lane hit
// for their parameter adjoints.  The 16
// geometry and density slots are summed over the wave (DPP and half-wave
// swaps) before one atomic per slot; the SH-coefficient slots, a per-ray
// constant times one scalar per (ray, Gaussian), are staged 16 Gaussians at a
// time and multiplied out on the matrix cores.  Two waves per SIMD: the
// tile's matrix operand and the staging buffer need the registers and LDS.

template <int NS, bool SG = false>
__global__ __launch_bounds__(kWave, 2) void k_backward(SceneDev s, ViewTable vt, MarchOpts op,
                                                    BwdIn in, LaunchShape ls) {
  __shared__ WaveMem M;
  __shared__ float sb[16 * kSbStride];   // staged S rows of the SH batch
  ShBatch shb;
  const int lane = threadIdx.x;
  const int n_active = uniform_int(s.counters[0]);
  const bool grid = !op.adaptive && op.ess != 2;
  bool first = true;
  for (;;) {
    int w;
    if (op.persistent) {
      w = pop_tile(ls.queue, vt.n_tiles, blockIdx.x & 7, lane);
      if (w < 0) break;
    } else {
      if (!first) break;
      w = xcd_block(blockIdx.x, gridDim.x);
      if (w >= vt.n_tiles) break;
    }
    first = false;

    const Pixel px = tile_pixel(vt, op, w, lane);
    const View &V = vt.v[px.view];
    const Ray r = make_ray(V, px.px, px.py);
    M.rdx[lane] = r.dx; M.rdy[lane] = r.dy; M.rdz[lane] = r.dz;
    M.rix[lane] = r.ix; M.riy[lane] = r.iy; M.riz[lane] = r.iz;
    const float tn = V.t_near, tf = V.t_far;
    float Y[16];
    sh_basis(op.sh_k, r.dx, r.dy, r.dz, Y);
    float Gc0 = 0, Gc1 = 0, Gc2 = 0, GCf = 0;
    if (px.valid) {
      const size_t q = 3 * (size_t)px.ray;
      Gc0 = in.grad_rgb[q];
      Gc1 = in.grad_rgb[q + 1];
      Gc2 = in.grad_rgb[q + 2];
      const float gT = in.grad_T ? in.grad_T[px.ray] : 0.0f;
      // G . C_fin + g_T T_fin; the colour still to come behind sample k is
      // C_fin - (prefix through k), kept as the running scalar GP = G . prefix
      GCf = Gc0 * in.rgb[q] + Gc1 * in.rgb[q + 1] + Gc2 * in.rgb[q + 2] + gT * in.T[px.ray];
    }
    // (the list arrays are free before the tile's first window)
    sh_batch_start(shb, sb, M.l_tin, Y, Gc0, Gc1, Gc2, lane);
    float GP = 0.0f;
    SegState ss;
    int n_closest = 0;   // closest-hit queries of this lane's ray so far
    WinRec rec;
    rec_start(rec, op, vt, w);
    ss.alive = px.valid;
    ss.pending = op.ess && px.valid;
    ss.seg_i = 0;
    ss.a = tn;
    ss.cl_lo = tn;
    const float dS = op.dt * (float)NS;
    Window win;
    const float seg_max = (float)NS * (op.adaptive ? op.dt_max : op.dt);
    win.len_min = (float)NS * (op.adaptive ? op.dt_min : op.dt);
    win.len = (float)op.window_segments * seg_max;
    win.len_max = fmaxf(8.0f * seg_max, 2.0f * win.len);
    win.valid = false;
    win.hi = -kInf;
    win.count = 0;
    win.kind = SRC_LIST;
    win.chunked = false;
    win.t.paused = false;
    win.t.z1 = n_active;
    int32_t dummy_nodes = 0, dummy_leaves = 0, dummy_windows = 0;
    float T = 1.0f;

    for (;;) {
      if (op.ess) closest_pass(s, op, n_active, r, tn, tf, dS, ss, ls.error_flag, nullptr, n_closest, px.ray);
      if (ss.alive) {
        const float a0 = grid ? fmaf((float)(ss.seg_i * NS), op.dt, tn) : ss.a;
        if (!(a0 < tf) || !(T > op.t_eps)) ss.alive = false;
      }
      if (ballot(ss.alive) == 0) break;
      float a = 0.0f, b = 0.0f, dt = op.dt;
      Samples sp;
      if (ss.alive) {
        if (!segment<NS>(op, grid, ss, tn, T, a, b, dt, sp)) {
          ss.alive = false;
          if (ls.error_flag) *ls.error_flag = 4;
        }
      }
      if (!ss.alive) { sp.t0 = 0.0f; sp.dt = 0.0f; }
      bool go;
      ensure_window<true>(s, op, M, r, lane, n_active, ss.alive, a, b, win, false, ls.error_flag,
                    dummy_nodes, dummy_leaves, dummy_windows, go, rec);
      const float a_min = wave_min(go ? a : kInf), b_max = wave_max(go ? b : -kInf);
      const float lo = go ? a : kInf, hi = go ? b : -kInf;
      // only G . W_k enters the adjoints, so pass A sums the Gaussians'
      // weights times G . c_l, one scalar per sample
      float sg[NS], GW[NS];
#pragma unroll
      for (int k = 0; k < NS; k++) { sg[k] = 0.0f; GW[k] = 0.0f; }
      int nhit = 0;
      // a replayed tile reads the forward's per-sample sums from its record;
      // pass A then only moves through the step's lists and marks
      const bool from_rec = op.replay_mode == 2 && rec.ok && op.sample_rec;

      // pass A: the forward's per-sample sums, in the forward's order
      do {
        const bool use_marks = rec_next_marks(rec, op, M, win.count, win.kind, lane, ls.error_flag);
        if (!from_rec)
        for_each_candidate<CAND_MARK>(win.kind, s, M, win.count, lane, a_min, b_max, n_active, r,
                                      [&](int j, const Gauss &g) {
        const bool want = go;
        const Chord c = chord(g, r);
        const bool hit = want & c.exists & (c.tin <= hi) & (c.tout >= lo);
        if (ballot(hit) == 0) return false;
        if (hit) {
          nhit++;
          float cr, cg, cb;
          colour(s.col, j, Y, cr, cg, cb);
          if constexpr (SG) sg_colour(s.sg, j, r.dx, r.dy, r.dz, cr, cg, cb);
          const float gc = fmaf(Gc0, cr, fmaf(Gc1, cg, Gc2 * cb));
          float wk[NS];
          sample_weights<NS>(g, c, sp, wk);
#pragma unroll
          for (int k = 0; k < NS; k++) {
            sg[k] += wk[k];
            GW[k] = fmaf(wk[k], gc, GW[k]);
          }
        }
        return true;
      }, use_marks);
      } while (next_chunk<true>(s, op, M, r, lane, n_active, go, a, b, win, false, ls.error_flag,
                            dummy_nodes, dummy_leaves, dummy_windows, rec));
      float best = kInf;
      if (from_rec)
        nhit = rec_get_samples<NS>(rec, op, go, Gc0, Gc1, Gc2, sg, GW, &best, lane, ls.error_flag) ? 1 : 0;

      // per-sample adjoints: dL/dsigma_k (into sg) and T_k phi_k (into GW);
      // dL/dW_k is G T_k phi_k
      const bool any = go && nhit > 0;
      if (any) {
#pragma unroll
        for (int k = 0; k < NS; k++) {
          float dsig = 0.0f, dW = 0.0f;
          if (sp.t(k) < tf && sg[k] > 0.0f) {
            const float x = sg[k] * dt;
            const float E = exp_neg(x);
            const float rs = __builtin_amdgcn_rcpf(sg[k]);
            const float alpha = one_minus_exp_neg(x);
            const float phi = alpha * rs;
            // d(alpha/sigma)/dsigma = dt^2 f'(x), f(x) = (1 - e^-x)/x
            const float dphi = x < 1e-2f
                ? dt * dt * (-0.5f + x * (1.0f / 3.0f - x * (0.125f - x * (1.0f / 30.0f))))
                : (x * E - alpha) * rs * rs;
            GP = fmaf(T * phi, GW[k], GP);
            dsig = T * dphi * GW[k] - dt * (GCf - GP);
            dW = T * phi;
            T *= E;
          }
          sg[k] = dsig;
          GW[k] = dW;
        }
      }

      // pass B: per-Gaussian adjoints
      if (ballot(any) != 0) {
        auto pass_b = [&](int j, const Gauss &g) {
          const bool want = any;
          float opx, opy, opz, dpx, dpy, dpz;
          ray_local(g, r, opx, opy, opz, dpx, dpy, dpz);
          const Chord c = chord(g, r);
          const bool hit = want & c.exists & (c.tin <= hi) & (c.tout >= lo);
          if (ballot(hit) == 0) return;
          float S = 0.0f;
          float v[16];
#pragma unroll
          for (int e2 = 0; e2 < 16; e2++) v[e2] = 0.0f;
          if (hit) {
            // the colour record's loads go out first: the sample weights and
            // the geometry terms below do not need them
            const ColRec rc = colour_load(s.col, j);
            float wk[NS];
            sample_weights<NS>(g, c, sp, wk);
            // closest-approach point in the local frame, and its world
            // offset from the mean
            const float pxl = fmaf(c.ts, dpx, opx), pyl = fmaf(c.ts, dpy, opy),
                        pzl = fmaf(c.ts, dpz, opz);
            const float Ps[3] = {fmaf(c.ts, r.dx, r.ox - g.mx), fmaf(c.ts, r.dy, r.oy - g.my),
                                 fmaf(c.ts, r.dz, r.oz - g.mz)};
            const float inv_sig = __builtin_amdgcn_rcpf(g.sig);
            float cr, cg, cb;
            colour_eval(rc, Y, cr, cg, cb);
            if constexpr (SG) sg_colour(s.sg, j, r.dx, r.dy, r.dz, cr, cg, cb);
            const float gc = fmaf(Gc0, cr, fmaf(Gc1, cg, Gc2 * cb));
            // dL/dw_k = dsigma_k + G.c_l T_k phi_k; dq_k = -w_k dL/dw_k / 2
            // moments over u_k = u_0 + k dt from sums over the sample index
            float ds = 0.0f, F1 = 0.0f, F2 = 0.0f;
#pragma unroll
            for (int k = 0; k < NS; k++) {
              const float wdw = wk[k] * fmaf(GW[k], gc, sg[k]);
              ds += wdw;
              F1 = fmaf((float)k, wdw, F1);
              F2 = fmaf((float)(k * k), wdw, F2);
              S = fmaf(wk[k], GW[k], S);
            }
            const float u0 = sp.t0 - c.ts;
            const float E1 = fmaf(u0, ds, sp.dt * F1);                         // sum wdw u
            const float E2 = fmaf(u0, fmaf(u0, ds, 2.0f * sp.dt * F1), sp.dt * sp.dt * F2);
            const float D0 = -0.5f * ds, D1 = -0.5f * E1, D2 = -0.5f * E2;
            // z_k = p + u_k d' with p = o' + t* d' (closest approach, local frame)
            const float Zs[3] = {fmaf(D0, pxl, D1 * dpx), fmaf(D0, pyl, D1 * dpy),
                                 fmaf(D0, pzl, D1 * dpz)};
            const float Us[3] = {fmaf(D1, pxl, D2 * dpx), fmaf(D1, pyl, D2 * dpy),
                                 fmaf(D1, pzl, D2 * dpz)};
            const float dd[3] = {r.dx, r.dy, r.dz};
            v[0] = Zs[0]; v[1] = Zs[1]; v[2] = Zs[2];
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
              for (int jj = 0; jj < 3; jj++) v[3 + 3 * i + jj] = fmaf(Zs[i], Ps[jj], Us[i] * dd[jj]);
            v[12] = fmaf(D0, pxl * pxl, fmaf(2.0f * D1, pxl * dpx, D2 * dpx * dpx));
            v[13] = fmaf(D0, pyl * pyl, fmaf(2.0f * D1, pyl * dpy, D2 * dpy * dpy));
            v[14] = fmaf(D0, pzl * pzl, fmaf(2.0f * D1, pzl * dpz, D2 * dpz * dpz));
            v[15] = ds * inv_sig;
          }
          // slots [0,16): geometry and density, summed over the wave; the SH
          // slots go through the matrix-core batch
          sb[shb.n * kSbStride + lane] = S;
          shb.id = lane == shb.n ? j : shb.id;
          const float mine = wave_sum_slots16(v, lane);
          if ((lane & 3) == 0) unsafeAtomicAdd(in.acc + (size_t)kAccFloats * j + (lane >> 2), mine);
          if constexpr (SG) sg_slots(s.sg, in.sgacc, j, hit ? S : 0.0f, Gc0, Gc1, Gc2, r, lane);
          if (++shb.n == 16) sh_batch_flush(shb, sb, in.acc, op.sh_k, lane);
        };
        // the list still holds the whole window, or the segment's last Z
        // chunk [zlast, end), its entries marked by pass A; a chunked segment
        // then visits [0, zlast): re-read from the record with the forward's
        // marks when replaying, else collected again
        const int zlast = win.chunked ? win.t.z0 : 0;
        const bool reread = win.chunked && zlast > 0 && rec.ok;
        uint32_t off = win.rec_first;
        int n_cur = win.count, kind_cur = win.kind;
        for (bool cur = true;; cur = false) {
          if (!cur) {
            if (!reread || off == win.rec_last || off == kWrecNone) break;
            uint32_t next, after;
            const int c = rec_load(op, M, off, lane, &next);
            n_cur = c > 0 ? c : 0;
            kind_cur = SRC_LIST;
            if (c < 0 || next == kWrecNone || !rec_load_marks(op, M, next, n_cur, lane, &after)) {
              if (ls.error_flag) *ls.error_flag = 5;
              break;
            }
            off = after;
          }
          for_each_candidate<CAND_FILTER>(kind_cur, s, M, n_cur, lane, a_min, b_max, n_active, r,
                                          pass_b);
        }
        if (win.chunked && zlast > 0 && !rec.ok) {
          first_chunk(s, M, r, lane, n_active, any, a, b, zlast, win, false, ls.error_flag,
                      dummy_nodes, dummy_leaves, dummy_windows);
          do for_each_candidate(win.kind, s, M, win.count, lane, a_min, b_max, n_active, r, pass_b);
          while (next_chunk<true>(s, op, M, r, lane, n_active, any, a, b, win, false, ls.error_flag,
                            dummy_nodes, dummy_leaves, dummy_windows, rec));
        }
      }

      // restart after an empty segment: from the list inside the window, else
      // through the closest-hit traversal (same decisions as the forward)
      const bool empty = go && nhit == 0;
      if (!from_rec && op.ess && win.kind == SRC_LIST && !win.chunked && ballot(empty)) {
        const float bmin = wave_min(empty ? b : kInf);
        for_each_candidate(SRC_LIST, s, M, win.count, lane, bmin, kInf, n_active, r,
                           [&](int j, const Gauss &g) {
          const bool want = empty;
          const Chord c = chord(g, r);
          if (want && c.exists && c.tout >= b && c.tin <= win.hi) best = fminf(best, fmaxf(c.tin, b));
        });
      }
      if (go) step_after(op, grid, nhit > 0, best, tn, dS, b, ss);
    }
    sh_batch_flush(shb, sb, in.acc, op.sh_k, lane);
  }
}

// ---------------------------------------------------------------------------
// Gradient finalisation: chain rule from the per-Gaussian accumulators to the
// user parameters (means, log-scales, quaternions through normalisation,
// density, SH), scattered to user order.
__global__ __launch_bounds__(256) void k_finalize(int64_t n, const int32_t *__restrict__ counters,
                                                  const uint32_t *__restrict__ perm,
                                                  const float *__restrict__ geom,
                                                  float *__restrict__ acc, int sh_k,
                                                  const float *__restrict__ aux,
                                                  float *__restrict__ gm, float *__restrict__ gl,
                                                  float *__restrict__ gq, float *__restrict__ gd,
                                                  float *__restrict__ gsh, int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t u = perm[i];
  // overwrite mode never reads the output buffers (they may hold anything)
  auto put = [accumulate](float &dst, float v) { dst = accumulate ? dst + v : v; };
  if (i >= counters[0]) {   // inactive Gaussian: zero gradient
    for (int k = 0; k < 3; k++) { put(gm[3 * u + k], 0.0f); put(gl[3 * u + k], 0.0f); }
    for (int k = 0; k < 4; k++) put(gq[4 * u + k], 0.0f);
    put(gd[u], 0.0f);
    for (int k = 0; k < 3 * sh_k; k++) put(gsh[(size_t)3 * sh_k * u + k], 0.0f);
    return;
  }
  float A[kAccFloats];
  float4 *accp = reinterpret_cast<float4 *>(acc + (size_t)kAccFloats * i);
  for (int k = 0; k < kAccFloats / 4; k++) {
    const float4 v = accp[k];
    A[4 * k] = v.x; A[4 * k + 1] = v.y; A[4 * k + 2] = v.z; A[4 * k + 3] = v.w;
    accp[k] = make_float4(0.f, 0.f, 0.f, 0.f);   // ready for the next backward
  }
  const float *G = geom + (size_t)kGeomFloats * i;
  float Z[3] = {A[0], A[1], A[2]};
  // dL/dmu = -2 M^T Z
  for (int jj = 0; jj < 3; jj++)
    put(gm[3 * u + jj], -2.0f * (G[G_M + jj] * Z[0] + G[G_M + 3 + jj] * Z[1] + G[G_M + 6 + jj] * Z[2]));
  // dL/dl_i = -2 sum z_i^2 dq
  for (int k = 0; k < 3; k++) put(gl[3 * u + k], -2.0f * A[12 + k]);
  // dL/dR_ji = 2 G'_ij / s_i
  const float *X = aux + (size_t)kAuxFloats * i;
  float dR[9];
  for (int ii = 0; ii < 3; ii++)
    for (int jj = 0; jj < 3; jj++) dR[3 * jj + ii] = 2.0f * A[3 + 3 * ii + jj] / X[ii];
  const float w = X[3], x = X[4], y = X[5], z = X[6], qn = X[7];
  float dq[4];
  dq[0] = 2.0f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
  dq[1] = 2.0f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.0f * x * dR[4] - w * dR[5] + z * dR[6] +
                  w * dR[7] - 2.0f * x * dR[8]);
  dq[2] = 2.0f * (-2.0f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] +
                  z * dR[7] - 2.0f * y * dR[8]);
  dq[3] = 2.0f * (-2.0f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.0f * z * dR[4] +
                  y * dR[5] + x * dR[6] + y * dR[7]);
  const float pr = dq[0] * w + dq[1] * x + dq[2] * y + dq[3] * z;
  const float qh[4] = {w, x, y, z};
  for (int k = 0; k < 4; k++) put(gq[4 * u + k], (dq[k] - pr * qh[k]) / qn);
  put(gd[u], A[15]);
  for (int m = 0; m < sh_k; m++)
    for (int ch = 0; ch < 3; ch++) {
      put(gsh[(size_t)3 * sh_k * u + 3 * m + ch], A[16 + 16 * ch + m]);
    }
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = i; k < n; k += stride) p[k] = v;
}

// ---------------------------------------------------------------------------

template <int NS>
static void fwd_dispatch(const SceneDev &s, const ViewTable &vt, const MarchOpts &op,
                         const FwdOut &out, const LaunchShape &ls, hipStream_t st) {
  if (out.dump_pix) k_forward<NS, true, false><<<ls.grid, kWave, 0, st>>>(s, vt, op, out, ls);
  else if (out.stats) k_forward<NS, false, true><<<ls.grid, kWave, 0, st>>>(s, vt, op, out, ls);
  else k_forward<NS, false, false><<<ls.grid, kWave, 0, st>>>(s, vt, op, out, ls);
}

// Lobed colour (spherical Gaussians): N_s = 8 only (checked by the host).
// The hit dump does not depend on colour and takes the plain kernel.
static void fwd_dispatch_sg(const SceneDev &s, const ViewTable &vt, const MarchOpts &op,
                            const FwdOut &out, const LaunchShape &ls, hipStream_t st) {
  if (out.dump_pix) k_forward<8, true, false><<<ls.grid, kWave, 0, st>>>(s, vt, op, out, ls);
  else if (out.stats) k_forward<8, false, true, true><<<ls.grid, kWave, 0, st>>>(s, vt, op, out, ls);
  else k_forward<8, false, false, true><<<ls.grid, kWave, 0, st>>>(s, vt, op, out, ls);
}

hipError_t launch_forward(const SceneDev &s, const ViewTable &vt, const MarchOpts &op,
                          const FwdOut &out, const LaunchShape &ls, hipStream_t st) {
  if (op.persistent) {
    hipError_t e = launch_fill(ls.queue, 8, 0u, st);
    if (e != hipSuccess) return e;
  }
  if (s.n_sg > 0) {
    if (op.n_s != 8) return hipErrorInvalidValue;
    fwd_dispatch_sg(s, vt, op, out, ls, st);
    return hipGetLastError();
  }
  switch (op.n_s) {
    case 1: fwd_dispatch<1>(s, vt, op, out, ls, st); break;
    case 2: fwd_dispatch<2>(s, vt, op, out, ls, st); break;
    case 4: fwd_dispatch<4>(s, vt, op, out, ls, st); break;
    case 8: fwd_dispatch<8>(s, vt, op, out, ls, st); break;
    case 16: fwd_dispatch<16>(s, vt, op, out, ls, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_backward(const SceneDev &s, const ViewTable &vt, const MarchOpts &op,
                           const BwdIn &in, const LaunchShape &ls, hipStream_t st) {
  if (op.persistent) {
    hipError_t e = launch_fill(ls.queue, 8, 0u, st);
    if (e != hipSuccess) return e;
  }
  if (s.n_sg > 0) {
    if (op.n_s != 8) return hipErrorInvalidValue;
    k_backward<8, true><<<ls.grid, kWave, 0, st>>>(s, vt, op, in, ls);
    return hipGetLastError();
  }
  switch (op.n_s) {
    case 1: k_backward<1><<<ls.grid, kWave, 0, st>>>(s, vt, op, in, ls); break;
    case 2: k_backward<2><<<ls.grid, kWave, 0, st>>>(s, vt, op, in, ls); break;
    case 4: k_backward<4><<<ls.grid, kWave, 0, st>>>(s, vt, op, in, ls); break;
    case 8: k_backward<8><<<ls.grid, kWave, 0, st>>>(s, vt, op, in, ls); break;
    case 16: k_backward<16><<<ls.grid, kWave, 0, st>>>(s, vt, op, in, ls); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_finalize_grads(const SceneDev &s, int sh_k, float *acc, float *g_means,
                                 float *g_log_scales, float *g_quats, float *g_density,
                                 float *g_sh, int accumulate, hipStream_t st) {
  const unsigned nb = (unsigned)((s.n + 255) / 256);
  k_finalize<<<nb, 256, 0, st>>>(s.n, s.counters, s.perm, s.geom, acc, sh_k, s.aux, g_means,
                                 g_log_scales, g_quats, g_density, g_sh, accumulate);
  return hipGetLastError();
}

// Lobe gradients to user order: per lobe, dL/da and dL/dlambda as summed;
// the axis through u = xi / |xi|: dL/dxi = lambda (h - (h.u) u) / |xi|.
// Absent lobes and inactive Gaussians get zeros.  Clears the accumulators.
__global__ __launch_bounds__(256) void k_finalize_sg(int64_t n, const int32_t *__restrict__ counters,
                                                     const uint32_t *__restrict__ perm,
                                                     const float *__restrict__ sg,
                                                     float *__restrict__ sgacc, int n_sg,
                                                     float *__restrict__ g_sg, int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t u = perm[i];
  const bool active = i < counters[0];
  for (int k = 0; k < n_sg; k++) {
    float out[kSgUserFloats] = {0, 0, 0, 0, 0, 0, 0};
    if (active) {
      const float *A = sgacc + (size_t)kSgAccFloats * i + kSgLobeFloats * k;
      const float *L = sg + (size_t)kSgFloats * i + kSgLobeFloats * k;
      if (L[7] > 0.0f) {
        const float h[3] = {A[4], A[5], A[6]};
        const float hu = h[0] * L[4] + h[1] * L[5] + h[2] * L[6];
        const float f = L[3] / L[7];
        out[0] = A[0]; out[1] = A[1]; out[2] = A[2];
        for (int e = 0; e < 3; e++) out[3 + e] = f * (h[e] - hu * L[4 + e]);
        out[6] = A[3];
      }
    }
    float *dst = g_sg + ((size_t)u * n_sg + k) * kSgUserFloats;
    for (int e = 0; e < kSgUserFloats; e++) dst[e] = accumulate ? dst[e] + out[e] : out[e];
  }
  if (active) {
    float4 *z = reinterpret_cast<float4 *>(sgacc + (size_t)kSgAccFloats * i);
    for (int e = 0; e < kSgAccFloats / 4; e++) z[e] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

hipError_t launch_finalize_sg(const SceneDev &s, float *sgacc, float *g_sg, int accumulate,
                              hipStream_t st) {
  const unsigned nb = (unsigned)((s.n + 255) / 256);
  k_finalize_sg<<<nb, 256, 0, st>>>(s.n, s.counters, s.perm, s.sg, sgacc, s.n_sg, g_sg, accumulate);
  return hipGetLastError();
}

// Densification statistic of one view (Sec. 3.5, Eq. 12).  The mean slots of
// the accumulators were zero when the view's backward started, so they hold
// that view's sum alone: its mean gradient is -2 M^T Z.  densify[user i] +=
// |mu - o| / f * |grad|, views += grad != 0.  The slots are then moved to
// zsum (the running sum over the call's views) and cleared for the next view;
// k_densify_restore puts the sum back before the chain rule.
__global__ __launch_bounds__(256) void k_densify(int64_t n, const int32_t *__restrict__ counters,
                                                 const uint32_t *__restrict__ perm,
                                                 const float *__restrict__ geom,
                                                 float *__restrict__ acc,
                                                 float *__restrict__ zsum, float ox, float oy,
                                                 float oz, float inv_focal,
                                                 float *__restrict__ densify,
                                                 int32_t *__restrict__ views) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || i >= counters[0]) return;
  const float *G = geom + (size_t)kGeomFloats * i;
  float z[3];
  for (int r = 0; r < 3; r++) {
    z[r] = acc[(size_t)kAccFloats * i + r];
    zsum[3 * i + r] += z[r];
    acc[(size_t)kAccFloats * i + r] = 0.0f;
  }
  float g2 = 0.0f;
  for (int c = 0; c < 3; c++) {
    const float gc = -2.0f * (G[G_M + c] * z[0] + G[G_M + 3 + c] * z[1] + G[G_M + 6 + c] * z[2]);
    g2 = fmaf(gc, gc, g2);
  }
  if (g2 > 0.0f) {
    const float ex = G[G_MU] - ox, ey = G[G_MU + 1] - oy, ez = G[G_MU + 2] - oz;
    const float alpha = sqrtf(ex * ex + ey * ey + ez * ez) * inv_focal;
    const uint32_t u = perm[i];
    densify[u] += alpha * sqrtf(g2);
    views[u] += 1;
  }
}

__global__ __launch_bounds__(256) void k_densify_restore(int64_t n, const int32_t *__restrict__ counters,
                                                         float *__restrict__ acc,
                                                         const float *__restrict__ zsum) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || i >= counters[0]) return;
  for (int r = 0; r < 3; r++) acc[(size_t)kAccFloats * i + r] = zsum[3 * i + r];
}

hipError_t launch_densify(const SceneDev &s, float *acc, float *zsum, float ox, float oy,
                          float oz, float focal, float *densify, int32_t *views, hipStream_t st) {
  const unsigned nb = (unsigned)((s.n + 255) / 256);
  k_densify<<<nb, 256, 0, st>>>(s.n, s.counters, s.perm, s.geom, acc, zsum, ox, oy, oz,
                                1.0f / focal, densify, views);
  return hipGetLastError();
}

hipError_t launch_densify_restore(const SceneDev &s, float *acc, const float *zsum, hipStream_t st) {
  const unsigned nb = (unsigned)((s.n + 255) / 256);
  k_densify_restore<<<nb, 256, 0, st>>>(s.n, s.counters, acc, zsum);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Statistics totals of one forward (int64, RGX_TOT_* order of the public
// header): per-block column sums of the per-ray counters, one atomic per
// column per block; the inactive Gaussians and the unrecorded tiles of the
// record are counted by the same launch.
enum { TOT_RAYS = 0, TOT_Q, TOT_P, TOT_SAMPLES, TOT_SEGMENTS, TOT_CLOSEST, TOT_NODES,
       TOT_BOX_ONLY, TOT_CHUNKED, TOT_INACTIVE, TOT_UNRECORDED, kNTot };

__global__ __launch_bounds__(256) void k_stat_totals(const int32_t *__restrict__ stats, int64_t rays,
                                                     int64_t n, const int32_t *__restrict__ counters,
                                                     const uint32_t *__restrict__ wrec_tile,
                                                     int64_t tiles, unsigned long long *totals) {
  constexpr int kCols = 8;
  const int cols[kCols] = {-1, ST_Q, ST_P, ST_SAMPLES, ST_SEGMENTS, ST_CLOSEST, ST_NODES, ST_BOX_ONLY};
  __shared__ unsigned long long red[kCols + 2][256];
  unsigned long long acc[kCols + 2];
#pragma unroll
  for (int c = 0; c < kCols + 2; c++) acc[c] = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rays; r += stride) {
    const int32_t *row = stats + (size_t)r * kNStat;
    acc[0] += 1;
#pragma unroll
    for (int c = 1; c < kCols; c++) acc[c] += (unsigned long long)(uint32_t)row[cols[c]];
    acc[kCols] += (unsigned long long)(uint32_t)row[ST_CHUNKED];
  }
  if (wrec_tile)
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tiles; t += stride)
      acc[kCols + 1] += wrec_tile[2 * t] == 1u ? 0ull : 1ull;
#pragma unroll
  for (int c = 0; c < kCols + 2; c++) red[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
#pragma unroll
      for (int c = 0; c < kCols + 2; c++) red[c][threadIdx.x] += red[c][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < kCols; c++) atomicAdd(&totals[c], red[c][0]);
    atomicAdd(&totals[TOT_CHUNKED], red[kCols][0]);
    atomicAdd(&totals[TOT_UNRECORDED], red[kCols + 1][0]);
    if (blockIdx.x == 0) atomicAdd(&totals[TOT_INACTIVE], (unsigned long long)(n - counters[0]));
  }
}

hipError_t launch_stat_totals(const int32_t *stats, int64_t rays, const SceneDev &s,
                              const uint32_t *wrec_tile, int64_t tiles, int64_t *totals,
                              hipStream_t st) {
  hipError_t e = launch_fill(totals, 2 * kNTot, 0u, st);
  if (e != hipSuccess) return e;
  const int64_t work = rays > tiles ? rays : tiles;
  int64_t nb = (work + 255) / 256;
  if (nb > 2048) nb = 2048;
  if (nb < 1) nb = 1;
  k_stat_totals<<<(unsigned)nb, 256, 0, st>>>(stats, rays, s.n, s.counters, wrec_tile, tiles,
                                              reinterpret_cast<unsigned long long *>(totals));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Whole-ray AABB false positives (Sec. 3.4, Eq. 6; minimal AABB of Supp. B)
// of listed pixels of one view: Gaussians whose minimal AABB mu +/- L,
// L_a = k sqrt(sum_m R_am^2 s_m^2), meets the ray over [t_n, t_end] while the
// ellipsoid's chord does not.  One thread per ray walks the binary LBVH with
// its own stack.  The node boxes are padded unions of padded leaf boxes, so
// they contain every minimal AABB below them and the walk misses none; the
// leaves then take the exact (unpadded) test.  Internal nodes lie at most 86
// levels deep (the Karras split positions grow strictly down the tree over
// the 63-bit key extended by a 23-bit index), and the walk pushes one child
// per level, so 96 stack entries always suffice.
constexpr int kFpStack = 96;

__global__ __launch_bounds__(256) void k_false_positives(SceneDev s, View V, const int32_t *__restrict__ pix,
                                                         int n_rays, const float *__restrict__ t_end,
                                                         int32_t *__restrict__ count,
                                                         int32_t *__restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_rays) return;
  const int n_active = s.counters[0];
  const int p = pix[i];
  const Ray r = make_ray(V, p % V.width, p / V.width);
  const float lo = V.t_near, hi = t_end[i];
  int fp = 0;
  auto leaf = [&](int j) {
    const Gauss g = with_origin(load_gauss_lane(s.geom, j), r.ox, r.oy, r.oz);
    const float *X = s.aux + (size_t)kAuxFloats * j;
    const float sx = X[0], sy = X[1], sz = X[2];
    const float w = X[3], x = X[4], y = X[5], z = X[6];
    // rows of R(q) for the unit quaternion (w, x, y, z)
    const float R[9] = {1.0f - 2.0f * (y * y + z * z), 2.0f * (x * y - w * z), 2.0f * (x * z + w * y),
                        2.0f * (x * y + w * z), 1.0f - 2.0f * (x * x + z * z), 2.0f * (y * z - w * x),
                        2.0f * (x * z - w * y), 2.0f * (y * z + w * x), 1.0f - 2.0f * (x * x + y * y)};
    const float k = sqrtf(g.k2);
    const float mu[3] = {g.mx, g.my, g.mz}, o[3] = {r.ox, r.oy, r.oz}, d[3] = {r.dx, r.dy, r.dz};
    float enter = lo, leave = hi;
#pragma unroll
    for (int a = 0; a < 3; a++) {
      const float e2 = R[3 * a] * R[3 * a] * sx * sx + R[3 * a + 1] * R[3 * a + 1] * sy * sy +
                       R[3 * a + 2] * R[3 * a + 2] * sz * sz;
      const float L = k * sqrtf(e2);
      const float ta = (mu[a] - L - o[a]) / d[a], tb = (mu[a] + L - o[a]) / d[a];
      enter = fmaxf(enter, fminf(ta, tb));
      leave = fminf(leave, fmaxf(ta, tb));
    }
    const Chord c = chord(g, r);
    const bool ell = c.exists && c.tin <= hi && c.tout >= lo;
    if (enter <= leave && !ell) fp++;
  };
  if (n_active == 1) {
    leaf(0);
  } else if (n_active > 1) {
    int stack[kFpStack];
    int sp = 0, node = 0;
    for (;;) {
      const vf4 *np = reinterpret_cast<const vf4 *>(s.nodes) + 4 * node;
      const vf4 a = np[0], b = np[1], c = np[2], d = np[3];
      const int cl = __float_as_int(a.w), cr = __float_as_int(b.w);
      const bool hL = cl != kNoChild && box_hit(a.x, a.y, a.z, b.x, b.y, b.z, r, lo, hi);
      const bool hR = cr != kNoChild && box_hit(c.x, c.y, c.z, d.x, d.y, d.z, r, lo, hi);
      int next = -1;
      if (hL) {
        if (cl < 0) leaf(~cl); else next = cl;
      }
      if (hR) {
        if (cr < 0) leaf(~cr);
        else if (next < 0) next = cr;
        else if (sp < kFpStack) stack[sp++] = cr;
        else { if (err) *err = 6; fp = -1; break; }
      }
      if (next >= 0) { node = next; continue; }
      if (sp == 0) break;
      node = stack[--sp];
    }
  }
  count[i] = fp;
}

hipError_t launch_false_positives(const SceneDev &s, const View &v, const int32_t *pix, int32_t n_rays,
                                  const float *t_end, int32_t *count, int32_t *error_flag,
                                  hipStream_t st) {
  if (n_rays <= 0) return hipSuccess;
  k_false_positives<<<(unsigned)((n_rays + 255) / 256), 256, 0, st>>>(s, v, pix, n_rays, t_end, count,
                                                                      error_flag);
  return hipGetLastError();
}

hipError_t launch_fill(void *p, int64_t n_words, uint32_t value, hipStream_t st) {
  if (n_words <= 0) return hipSuccess;
  int64_t blocks = (n_words + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_fill_u32<<<(unsigned)blocks, 256, 0, st>>>((uint32_t *)p, n_words, value);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t st) {
  return launch_fill(p, n, __builtin_bit_cast(uint32_t, v), st);
}

}  // namespace rgx

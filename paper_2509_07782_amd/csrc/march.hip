// Forward and backward ray marching through the Gaussian field (Sec. 3.1
// Eq. 1-3; Sec. 3.2 Algorithm 1, Eq. 4-5).
//
// Execution model: one wave64 owns one ray tile (64 rays).  The wave walks the
// LBVH as a packet: a node is entered when any active lane's ray meets one of
// its child boxes over that lane's own interval, and the traversal stack is
// wave-uniform, held one entry per lane in two VGPRs (writelane/readlane).
// Node and Gaussian records are read at wave-uniform addresses through the
// scalar cache.  Leaves are met in left-to-right (= Z order) order whatever
// subset of the tree a packet visits, so every lane accumulates its samples
// in the same order under the BVH, under brute force, for any tile shape and
// ray order, which makes those images bit-identical.
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

// Geometry of one Gaussian (wave-uniform, from the scalar cache).
struct Gauss {
  float mx, my, mz, k2;
  float m[9];
  float sig, l2sig;
};

__device__ __forceinline__ Gauss load_gauss(const float *geom, int j) {
  cfloat4p p = as_const4(geom) + 4 * j;
  const vf4 a = p[0], b = p[1], c = p[2], d = p[3];
  Gauss g;
  g.mx = a.x; g.my = a.y; g.mz = a.z; g.k2 = a.w;
  g.m[0] = b.x; g.m[1] = b.y; g.m[2] = b.z; g.m[3] = b.w;
  g.m[4] = c.x; g.m[5] = c.y; g.m[6] = c.z; g.m[7] = c.w;
  g.m[8] = d.x; g.sig = d.y; g.l2sig = d.z;
  return g;
}

// Ray / ellipsoid {q <= k^2}: q(t) = A (t - t*)^2 + h^2 about the point of
// closest approach; the chord is t* -/+ sqrt((k^2 - h^2) / A).
struct Chord {
  float A, ts, h2, tin, tout;
  bool exists;
};

__device__ __forceinline__ void ray_local(const Gauss &g, const Ray &r, float &opx, float &opy,
                                          float &opz, float &dpx, float &dpy, float &dpz) {
  const float ex = r.ox - g.mx, ey = r.oy - g.my, ez = r.oz - g.mz;
  opx = fmaf(g.m[0], ex, fmaf(g.m[1], ey, g.m[2] * ez));
  opy = fmaf(g.m[3], ex, fmaf(g.m[4], ey, g.m[5] * ez));
  opz = fmaf(g.m[6], ex, fmaf(g.m[7], ey, g.m[8] * ez));
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
  c.ts = -B / c.A;
  const float px = fmaf(c.ts, dpx, opx), py = fmaf(c.ts, dpy, opy), pz = fmaf(c.ts, dpz, opz);
  c.h2 = fmaf(px, px, fmaf(py, py, pz * pz));
  c.exists = c.h2 <= g.k2;
  const float w = sqrtf(fmaxf(g.k2 - c.h2, 0.0f) / c.A);
  c.tin = c.ts - w;
  c.tout = c.ts + w;
  return c;
}

// Colour of a Gaussian at the lane's direction: c = sum_m f_m Y_m.
__device__ __forceinline__ void colour(const float *col, int j, int col_stride, int sh_k,
                                       const float *Y, float &cr, float &cg, float &cb) {
  cfloat4p p = as_const4(col) + (size_t)(col_stride >> 2) * j;
  float acc[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int q = 0; q < 12; q++) {
    if (4 * q < 3 * sh_k) {
      const vf4 f = p[q];
      const float fv[4] = {f.x, f.y, f.z, f.w};
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const int flat = 4 * q + e;
        if (flat < 3 * sh_k) acc[flat % 3] = fmaf(fv[e], Y[flat / 3], acc[flat % 3]);
      }
    }
  }
  cr = acc[0]; cg = acc[1]; cb = acc[2];
}

// Wave-uniform DFS stack, entry i held by lane i of s0 (i < 64) or s1.
struct WaveStack {
  int s0 = 0, s1 = 0, sp = 0, lane = 0;
  __device__ __forceinline__ bool push(int v) {
    if (sp < 64) s0 = lane == sp ? v : s0;
    else if (sp < 128) s1 = lane == sp - 64 ? v : s1;
    else return false;
    sp++;
    return true;
  }
  __device__ __forceinline__ int pop() {
    sp--;
    return sp < 64 ? __builtin_amdgcn_readlane(s0, sp) : __builtin_amdgcn_readlane(s1, sp - 64);
  }
};

// Packet traversal in left-to-right leaf order.  `lo`/`hi` are per-lane
// interval references (hi may shrink inside `leaf`).  Leaves whose box meets
// some lane's interval are passed to leaf(j) with j wave-uniform.
template <class Leaf>
__device__ __forceinline__ void traverse(const SceneDev &s, int n_active, const Ray &r,
                                         const float &lo, const float &hi, int32_t *err,
                                         Leaf &&leaf) {
  if (n_active <= 0) return;
  WaveStack st;
  st.lane = __lane_id();
  int node = 0;
  const int n_inner = n_active > 1 ? n_active - 1 : 1;
  // a valid tree visits each of its n_inner nodes at most once
  for (int visits = 0;; visits++) {
    if (visits > n_inner) { if (err) *err = 2; return; }
    cfloat4p np = as_const4(s.nodes) + 4 * node;
    const vf4 a = np[0], b = np[1], c = np[2], d = np[3];
    const int cl = __float_as_int(a.w), cr = __float_as_int(b.w);
    // child references must stay inside the structure
    const bool bad = (cl >= 0 ? cl >= n_inner : ~cl >= n_active) ||
                     (cr != kNoChild && (cr >= 0 ? cr >= n_inner : ~cr >= n_active));
    if (bad) { if (err) *err = 3; return; }
    bool hl = ballot(box_hit(a.x, a.y, a.z, b.x, b.y, b.z, r, lo, hi)) != 0;
    bool hr = cr != kNoChild && ballot(box_hit(c.x, c.y, c.z, d.x, d.y, d.z, r, lo, hi)) != 0;
    if (hl && cl < 0) { leaf(~cl); hl = false; }
    if (hr && cr < 0 && !hl) { leaf(~cr); hr = false; }
    if (hl) {
      if (hr && !st.push(cr)) { if (err) *err = 1; return; }
      node = cl;
      continue;
    }
    if (hr) { node = cr; continue; }
    bool found = false;
    while (st.sp > 0) {
      const int v = st.pop();
      if (v < 0) { leaf(~v); continue; }
      node = v;
      found = true;
      break;
    }
    if (!found) return;
  }
}

// Brute force: every active Gaussian in Z order (the hit-set reference).
template <class Leaf>
__device__ __forceinline__ void brute_all(int n_active, Leaf &&leaf) {
  for (int j = 0; j < n_active; j++) leaf(j);
}

template <class Leaf>
__device__ __forceinline__ void for_each_candidate(const SceneDev &s, const MarchOpts &op,
                                                   int n_active, const Ray &r, const float &lo,
                                                   const float &hi, int32_t *err, Leaf &&leaf) {
  if (op.brute_force) brute_all(n_active, leaf);
  else traverse(s, n_active, r, lo, hi, err, leaf);
}

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

__device__ __forceinline__ Ray make_ray(const View &V, int px, int py) {
  Ray r;
  r.ox = V.c2w[3]; r.oy = V.c2w[7]; r.oz = V.c2w[11];
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

template <int NS>
__device__ __forceinline__ void sample_positions(bool grid, int seg_i, float a, float dt, float tn,
                                                 float *t) {
#pragma unroll
  for (int k = 0; k < NS; k++)
    t[k] = grid ? fmaf((float)(seg_i * NS + k) + 0.5f, dt, tn) : fmaf((float)k + 0.5f, dt, a);
}

// Eq. 5 with d_i = a (unit direction from the camera centre).
__device__ __forceinline__ float adaptive_dt(const MarchOpts &op, float a, float T) {
  const float base = fmaxf(a * op.inv_beta, op.dt_min);
  const float v = base * exp2f(-__log2f(T) * (1.0f / 3.0f));
  return v < op.dt_max ? v : op.dt_max;
}

// Per-lane segment state shared by forward and backward.
struct SegState {
  bool alive, pending;
  int seg_i;
  float a, cl_lo;
};

// Closest hit (Alg. 1 ClosestHit, Eq. 4) for the lanes with `pending` set:
// min over Gaussians whose chord meets [cl_lo, t_far] of max(t_in, cl_lo).
__device__ __forceinline__ void closest_pass(const SceneDev &s, const MarchOpts &op, int n_active,
                                             const Ray &r, float tn, float tf, float dS,
                                             SegState &ss, int32_t *err, int32_t *st_closest) {
  if (ballot(ss.pending) == 0) return;
  float lo = ss.pending ? ss.cl_lo : kInf;
  float hi = ss.pending ? tf : -kInf;
  float best = kInf;
  for_each_candidate(s, op, n_active, r, lo, hi, err, [&](int j) {
    const Gauss g = load_gauss(s.geom, j);
    const Chord c = chord(g, r);
    if (c.exists && c.tin <= hi && c.tout >= lo) {
      best = fminf(best, fmaxf(c.tin, lo));
      hi = fminf(hi, best);
    }
  });
  if (ss.pending) {
    if (st_closest) (*st_closest)++;
    if (!(best < kInf)) ss.alive = false;
    else if (!op.adaptive && op.ess == 1) {
      const int j = (int)floorf((best - tn) / dS);
      ss.seg_i = max(ss.seg_i, j);
    } else ss.a = best;
    ss.pending = false;
  }
}

// ---------------------------------------------------------------------------
// Forward kernel (and the hit-dump variant).

template <int NS, bool DUMP>
__global__ __launch_bounds__(kBlock) void k_forward(SceneDev s, ViewTable vt, MarchOpts op,
                                                    FwdOut out, LaunchShape ls) {
  const int lane = threadIdx.x & 63, wib = threadIdx.x >> 6;
  const int n_active = uniform_int(s.counters[0]);
  const bool grid = !op.adaptive && op.ess != 2;
  const bool stats = out.stats != nullptr;
  bool first = true;
  for (;;) {
    int w;
    if (op.persistent) {
      w = pop_tile(ls.queue, vt.n_tiles, blockIdx.x & 7, lane);
      if (w < 0) break;
    } else {
      if (!first) break;
      w = xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + wib;
      if (w >= vt.n_tiles) break;
    }
    first = false;

    Pixel px;
    View V;
    int dump_slot = 0;
    if (DUMP) {
      V = vt.v[0];
      dump_slot = w * 64 + lane;
      px.valid = dump_slot < out.dump_n;
      const int pix = px.valid ? out.dump_pix[dump_slot] : 0;
      px.px = pix % V.width; px.py = pix / V.width; px.ray = dump_slot;
    } else {
      px = tile_pixel(vt, op, w, lane);
      V = vt.v[px.view];
    }
    const Ray r = make_ray(V, px.px, px.py);
    const float tn = V.t_near, tf = V.t_far;
    float Y[16];
    sh_basis(op.sh_k, r.dx, r.dy, r.dz, Y);

    SegState ss;
    ss.alive = px.valid;
    ss.pending = op.ess && px.valid;
    ss.seg_i = 0;
    ss.a = tn;
    ss.cl_lo = tn;
    const float dS = op.dt * (float)NS;
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    int32_t cnt[kNStatUsed] = {0, 0, 0, 0, 0, 0};
    float prev_a = -kInf, prev_b = -kInf;
    int n_dump = 0;

    for (;;) {
      if (op.ess)
        closest_pass(s, op, n_active, r, tn, tf, dS, ss, ls.error_flag,
                     stats ? &cnt[ST_CLOSEST] : nullptr);
      float a = 0.0f, b = 0.0f, dt = op.dt;
      if (ss.alive) {
        a = grid ? fmaf((float)(ss.seg_i * NS), op.dt, tn) : ss.a;
        if (!(a < tf) || !(T > op.t_eps)) ss.alive = false;
      }
      if (ballot(ss.alive) == 0) break;
      float lo = kInf, hi = -kInf;
      if (ss.alive) {
        if (op.adaptive) dt = adaptive_dt(op, a, T);
        b = grid ? fmaf((float)((ss.seg_i + 1) * NS), op.dt, tn) : fmaf((float)NS, dt, a);
        lo = a;
        hi = b;
        if (!(b > a)) {   // no progress possible in FP32: stop this ray
          ss.alive = false;
          lo = kInf;
          hi = -kInf;
          if (ls.error_flag) *ls.error_flag = 4;
        }
      }
      float ts[NS];
      sample_positions<NS>(grid, ss.seg_i, a, dt, tn, ts);
      float sg[NS], W0[NS], W1[NS], W2[NS];
#pragma unroll
      for (int k = 0; k < NS; k++) { sg[k] = 0.0f; W0[k] = W1[k] = W2[k] = 0.0f; }
      int nhit = 0;

      for_each_candidate(s, op, n_active, r, lo, hi, ls.error_flag, [&](int j) {
        const Gauss g = load_gauss(s.geom, j);
        const Chord c = chord(g, r);
        const bool hit = c.exists && c.tin <= hi && c.tout >= lo;
        if (stats) {
          const float *bx = s.aabb + 6 * (size_t)j;
          const bool boxed = box_hit(bx[0], bx[1], bx[2], bx[3], bx[4], bx[5], r, lo, hi);
          if (boxed && !hit) cnt[ST_BOX_ONLY]++;
        }
        if (ballot(hit) == 0) return;
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
          float cr, cg, cb;
          colour(s.col, j, op.col_stride, op.sh_k, Y, cr, cg, cb);
#pragma unroll
          for (int k = 0; k < NS; k++) {
            const float u = ts[k] - c.ts;
            const float q = fmaf(c.A * u, u, c.h2);
            const float wv = exp2f(fmaf(-q, kHalfLog2e, g.l2sig));
            const float w = q <= g.k2 ? wv : 0.0f;
            sg[k] += w;
            W0[k] = fmaf(w, cr, W0[k]);
            W1[k] = fmaf(w, cg, W1[k]);
            W2[k] = fmaf(w, cb, W2[k]);
          }
        }
      });

      if (ss.alive) {
        if (nhit == 0) {
          if (op.ess) { ss.pending = true; ss.cl_lo = b; ss.seg_i += 1; }
          else if (grid) ss.seg_i += 1;
          else ss.a = b;
        } else {
          if (stats) { cnt[ST_SEGMENTS]++; cnt[ST_P] += nhit; }
#pragma unroll
          for (int k = 0; k < NS; k++) {
            if (ts[k] < tf) {
              if (stats) cnt[ST_SAMPLES]++;
              if (sg[k] > 0.0f) {
                const float x = sg[k] * dt;
                const float alpha = one_minus_exp_neg(x);
                const float f = T * (alpha / sg[k]);
                C0 = fmaf(f, W0[k], C0);
                C1 = fmaf(f, W1[k], C1);
                C2 = fmaf(f, W2[k], C2);
                T *= __expf(-x);
              }
            }
          }
          prev_a = a;
          prev_b = b;
          if (grid) ss.seg_i += 1;
          else ss.a = b;
        }
      }
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
// Backward kernel.

// Reduce-scatter of 64 values across the wave: afterwards lane L holds the sum
// over all lanes of v[L].
__device__ __forceinline__ float wave_reduce_scatter64(float *v, int lane) {
#pragma unroll
  for (int h = 32; h >= 1; h >>= 1) {
    const bool up = (lane & h) != 0;
#pragma unroll
    for (int i = 0; i < h; i++) {
      const float keep = up ? v[i + h] : v[i];
      const float send = up ? v[i] : v[i + h];
      v[i] = keep + __shfl_xor(send, h, 64);
    }
  }
  return v[0];
}

constexpr int kListCap = 512;   // per-wave LDS list of a segment's Gaussians

template <int NS>
__global__ __launch_bounds__(kBlock) void k_backward(SceneDev s, ViewTable vt, MarchOpts op,
                                                     BwdIn in, LaunchShape ls) {
  __shared__ int32_t list_mem[kWavesPerBlock][kListCap];
  const int lane = threadIdx.x & 63, wib = threadIdx.x >> 6;
  int32_t *list = list_mem[wib];
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
      w = xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + wib;
      if (w >= vt.n_tiles) break;
    }
    first = false;

    const Pixel px = tile_pixel(vt, op, w, lane);
    const View &V = vt.v[px.view];
    const Ray r = make_ray(V, px.px, px.py);
    const float tn = V.t_near, tf = V.t_far;
    float Y[16];
    sh_basis(op.sh_k, r.dx, r.dy, r.dz, Y);
    float Gc0 = 0, Gc1 = 0, Gc2 = 0, Cf0 = 0, Cf1 = 0, Cf2 = 0, gT = 0, Tfin = 0;
    if (px.valid) {
      Gc0 = in.grad_rgb[3 * (size_t)px.ray];
      Gc1 = in.grad_rgb[3 * (size_t)px.ray + 1];
      Gc2 = in.grad_rgb[3 * (size_t)px.ray + 2];
      Cf0 = in.rgb[3 * (size_t)px.ray];
      Cf1 = in.rgb[3 * (size_t)px.ray + 1];
      Cf2 = in.rgb[3 * (size_t)px.ray + 2];
      Tfin = in.T[px.ray];
      gT = in.grad_T ? in.grad_T[px.ray] : 0.0f;
    }
    // G . (C_fin - P_k) + g_T T_fin, kept as a running scalar: GC - G.P
    const float GCf = Gc0 * Cf0 + Gc1 * Cf1 + Gc2 * Cf2 + gT * Tfin;
    float GP = 0.0f;
    SegState ss;
    ss.alive = px.valid;
    ss.pending = op.ess && px.valid;
    ss.seg_i = 0;
    ss.a = tn;
    ss.cl_lo = tn;
    const float dS = op.dt * (float)NS;
    float T = 1.0f;

    for (;;) {
      if (op.ess) closest_pass(s, op, n_active, r, tn, tf, dS, ss, ls.error_flag, nullptr);
      float a = 0.0f, b = 0.0f, dt = op.dt;
      if (ss.alive) {
        a = grid ? fmaf((float)(ss.seg_i * NS), op.dt, tn) : ss.a;
        if (!(a < tf) || !(T > op.t_eps)) ss.alive = false;
      }
      if (ballot(ss.alive) == 0) break;
      float lo = kInf, hi = -kInf;
      if (ss.alive) {
        if (op.adaptive) dt = adaptive_dt(op, a, T);
        b = grid ? fmaf((float)((ss.seg_i + 1) * NS), op.dt, tn) : fmaf((float)NS, dt, a);
        lo = a;
        hi = b;
        if (!(b > a)) {   // no progress possible in FP32: stop this ray
          ss.alive = false;
          lo = kInf;
          hi = -kInf;
          if (ls.error_flag) *ls.error_flag = 4;
        }
      }
      float ts[NS];
      sample_positions<NS>(grid, ss.seg_i, a, dt, tn, ts);
      float sg[NS], W0[NS], W1[NS], W2[NS];
#pragma unroll
      for (int k = 0; k < NS; k++) { sg[k] = 0.0f; W0[k] = W1[k] = W2[k] = 0.0f; }
      int nhit = 0;
      int nlist = 0;

      // pass A: the forward's per-sample sums, in the forward's order
      for_each_candidate(s, op, n_active, r, lo, hi, ls.error_flag, [&](int j) {
        const Gauss g = load_gauss(s.geom, j);
        const Chord c = chord(g, r);
        const bool hit = c.exists && c.tin <= hi && c.tout >= lo;
        if (ballot(hit) == 0) return;
        if (nlist < kListCap && lane == 0) list[nlist] = j;
        nlist++;
        if (hit) {
          nhit++;
          float cr, cg, cb;
          colour(s.col, j, op.col_stride, op.sh_k, Y, cr, cg, cb);
#pragma unroll
          for (int k = 0; k < NS; k++) {
            const float u = ts[k] - c.ts;
            const float q = fmaf(c.A * u, u, c.h2);
            const float wv = exp2f(fmaf(-q, kHalfLog2e, g.l2sig));
            const float w = q <= g.k2 ? wv : 0.0f;
            sg[k] += w;
            W0[k] = fmaf(w, cr, W0[k]);
            W1[k] = fmaf(w, cg, W1[k]);
            W2[k] = fmaf(w, cb, W2[k]);
          }
        }
      });

      __builtin_amdgcn_wave_barrier();
      // per-sample adjoints dL/dsigma_k (reusing sg) and dL/dW_k (reusing W)
      bool any = false;
      if (ss.alive && nhit > 0) {
        any = true;
#pragma unroll
        for (int k = 0; k < NS; k++) {
          float dsig = 0.0f, dW = 0.0f;
          if (ts[k] < tf && sg[k] > 0.0f) {
            const float x = sg[k] * dt;
            const float E = __expf(-x);
            const float alpha = one_minus_exp_neg(x);
            const float phi = alpha / sg[k];
            // d(alpha/sigma)/dsigma = dt^2 f'(x), f(x) = (1 - e^-x)/x
            const float dphi = x < 1e-2f
                ? dt * dt * (-0.5f + x * (1.0f / 3.0f - x * (0.125f - x * (1.0f / 30.0f))))
                : (x * E - alpha) / (sg[k] * sg[k]);
            const float GW = Gc0 * W0[k] + Gc1 * W1[k] + Gc2 * W2[k];
            GP = fmaf(T * phi, GW, GP);
            dsig = T * dphi * GW - dt * (GCf - GP);
            dW = T * phi;
            T *= E;
          }
          sg[k] = dsig;
          W0[k] = dW * Gc0;
          W1[k] = dW * Gc1;
          W2[k] = dW * Gc2;
        }
      }

      // pass B: per-Gaussian gradient contributions, wave-reduced, then atomics
      if (ballot(any) != 0) {
        const int nl = nlist;
        auto leafB = [&](int j) {
          const Gauss g = load_gauss(s.geom, j);
          float opx, opy, opz, dpx, dpy, dpz;
          ray_local(g, r, opx, opy, opz, dpx, dpy, dpz);
          const Chord c = chord(g, r);
          const bool hit = any && c.exists && c.tin <= hi && c.tout >= lo;
          if (ballot(hit) == 0) return;
          float v[kAccFloats];
#pragma unroll
          for (int e = 0; e < kAccFloats; e++) v[e] = 0.0f;
          if (hit) {
            float cr, cg, cb;
            colour(s.col, j, op.col_stride, op.sh_k, Y, cr, cg, cb);
            float D0 = 0.0f, D1 = 0.0f, D2 = 0.0f, dc0 = 0.0f, dc1 = 0.0f, dc2 = 0.0f, ds = 0.0f;
#pragma unroll
            for (int k = 0; k < NS; k++) {
              const float u = ts[k] - c.ts;
              const float q = fmaf(c.A * u, u, c.h2);
              const float wv = exp2f(fmaf(-q, kHalfLog2e, g.l2sig));
              const float w = q <= g.k2 ? wv : 0.0f;
              const float dw = sg[k] + W0[k] * cr + W1[k] * cg + W2[k] * cb;
              const float wdw = w * dw;
              ds += wdw;
              const float dq = -0.5f * wdw;
              D0 += dq;
              D1 = fmaf(dq, u, D1);
              D2 = fmaf(dq * u, u, D2);
              dc0 = fmaf(w, W0[k], dc0);
              dc1 = fmaf(w, W1[k], dc1);
              dc2 = fmaf(w, W2[k], dc2);
            }
            // z_k = p + u_k d' with p = o' + t* d' (closest approach, local frame)
            const float pxl = fmaf(c.ts, dpx, opx), pyl = fmaf(c.ts, dpy, opy),
                        pzl = fmaf(c.ts, dpz, opz);
            const float Z0 = fmaf(D0, pxl, D1 * dpx), Z1 = fmaf(D0, pyl, D1 * dpy),
                        Z2 = fmaf(D0, pzl, D1 * dpz);
            const float U0 = fmaf(D1, pxl, D2 * dpx), U1 = fmaf(D1, pyl, D2 * dpy),
                        U2 = fmaf(D1, pzl, D2 * dpz);
            // world offset of the closest-approach point from the mean
            const float P0 = fmaf(c.ts, r.dx, r.ox - g.mx), P1 = fmaf(c.ts, r.dy, r.oy - g.my),
                        P2 = fmaf(c.ts, r.dz, r.oz - g.mz);
            v[0] = Z0; v[1] = Z1; v[2] = Z2;
            const float Zs[3] = {Z0, Z1, Z2}, Us[3] = {U0, U1, U2}, Ps[3] = {P0, P1, P2},
                        ds3[3] = {r.dx, r.dy, r.dz};
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
              for (int jj = 0; jj < 3; jj++) v[3 + 3 * i + jj] = fmaf(Zs[i], Ps[jj], Us[i] * ds3[jj]);
            v[12] = fmaf(D0, pxl * pxl, fmaf(2.0f * D1, pxl * dpx, D2 * dpx * dpx));
            v[13] = fmaf(D0, pyl * pyl, fmaf(2.0f * D1, pyl * dpy, D2 * dpy * dpy));
            v[14] = fmaf(D0, pzl * pzl, fmaf(2.0f * D1, pzl * dpz, D2 * dpz * dpz));
            v[15] = ds / g.sig;
#pragma unroll
            for (int m = 0; m < 16; m++) {
              if (m < op.sh_k) {
                v[16 + 3 * m] = Y[m] * dc0;
                v[17 + 3 * m] = Y[m] * dc1;
                v[18 + 3 * m] = Y[m] * dc2;
              }
            }
          }
          const float tot = wave_reduce_scatter64(v, lane);
          if (lane < 16 + 3 * op.sh_k)
            unsafeAtomicAdd(in.acc + (size_t)kAccFloats * j + lane, tot);
        };
        if (nl <= kListCap) {
          for (int e = 0; e < nl; e++) leafB(uniform_int(list[e]));
        } else {
          for_each_candidate(s, op, n_active, r, lo, hi, ls.error_flag, leafB);
        }
      }

      if (ss.alive) {
        if (nhit == 0) {
          if (op.ess) { ss.pending = true; ss.cl_lo = b; ss.seg_i += 1; }
          else if (grid) ss.seg_i += 1;
          else ss.a = b;
        } else {
          if (grid) ss.seg_i += 1;
          else ss.a = b;
        }
      }
    }
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
  const float keep = accumulate ? 1.0f : 0.0f;
  if (i >= counters[0]) {   // inactive Gaussian: zero gradient
    for (int k = 0; k < 3; k++) { gm[3 * u + k] *= keep; gl[3 * u + k] *= keep; }
    for (int k = 0; k < 4; k++) gq[4 * u + k] *= keep;
    gd[u] *= keep;
    for (int k = 0; k < 3 * sh_k; k++) gsh[(size_t)3 * sh_k * u + k] *= keep;
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
    gm[3 * u + jj] = fmaf(keep, gm[3 * u + jj],
                          -2.0f * (G[G_M + jj] * Z[0] + G[G_M + 3 + jj] * Z[1] + G[G_M + 6 + jj] * Z[2]));
  // dL/dl_i = -2 sum z_i^2 dq
  for (int k = 0; k < 3; k++) gl[3 * u + k] = fmaf(keep, gl[3 * u + k], -2.0f * A[12 + k]);
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
  for (int k = 0; k < 4; k++) gq[4 * u + k] = fmaf(keep, gq[4 * u + k], (dq[k] - pr * qh[k]) / qn);
  gd[u] = fmaf(keep, gd[u], A[15]);
  for (int k = 0; k < 3 * sh_k; k++)
    gsh[(size_t)3 * sh_k * u + k] = fmaf(keep, gsh[(size_t)3 * sh_k * u + k], A[16 + k]);
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
  if (out.dump_pix) k_forward<NS, true><<<ls.grid, kBlock, 0, st>>>(s, vt, op, out, ls);
  else k_forward<NS, false><<<ls.grid, kBlock, 0, st>>>(s, vt, op, out, ls);
}

hipError_t launch_forward(const SceneDev &s, const ViewTable &vt, const MarchOpts &op,
                          const FwdOut &out, const LaunchShape &ls, hipStream_t st) {
  if (op.persistent) {
    hipError_t e = launch_fill(ls.queue, 8, 0u, st);
    if (e != hipSuccess) return e;
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
  switch (op.n_s) {
    case 1: k_backward<1><<<ls.grid, kBlock, 0, st>>>(s, vt, op, in, ls); break;
    case 2: k_backward<2><<<ls.grid, kBlock, 0, st>>>(s, vt, op, in, ls); break;
    case 4: k_backward<4><<<ls.grid, kBlock, 0, st>>>(s, vt, op, in, ls); break;
    case 8: k_backward<8><<<ls.grid, kBlock, 0, st>>>(s, vt, op, in, ls); break;
    case 16: k_backward<16><<<ls.grid, kBlock, 0, st>>>(s, vt, op, in, ls); break;
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

// Acceleration-structure build: per-Gaussian preprocessing, Z-order (Morton)
// keys, a stable LSD radix sort, the Z-ordered pack, and a Karras LBVH whose
// node boxes come from range unions over a segment tree of the leaf boxes.  Every size follows from N on the host; the number of
// active Gaussians stays on the device, so the whole build is asynchronous.
#include "common.hpp"
#include "internal.hpp"

namespace rgx {

// ---------------------------------------------------------------------------
// Order-preserving float <-> uint32 map for atomic min/max of floats.
__device__ __forceinline__ uint32_t f2ord(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__global__ void k_build_init(uint32_t *bounds, int32_t *counters) {
  int t = threadIdx.x;
  if (t < 3) bounds[t] = 0xffffffffu;        // min
  else if (t < 6) bounds[t] = 0u;            // max
  if (t < 8) counters[t] = 0;
}

// Per Gaussian (user order): Sec. 3.1 Eq. 1 and the sigma_eps level-set
// ellipsoid of Supp. B.  Writes the geometry record, the padded AABB and an
// active flag; accumulates the bounds of the active means.
__global__ __launch_bounds__(256) void k_preprocess(int64_t n, const float *__restrict__ means,
                                                    const float *__restrict__ log_scales,
                                                    const float *__restrict__ quats,
                                                    const float *__restrict__ density,
                                                    float sigma_eps, float *__restrict__ geom,
                                                    float *__restrict__ aabb,
                                                    float *__restrict__ aux,
                                                    uint8_t *__restrict__ active,
                                                    uint32_t *__restrict__ bounds,
                                                    int32_t *__restrict__ counters) {
  __shared__ uint32_t sb[6];
  __shared__ int32_t scount;
  if (threadIdx.x < 3) sb[threadIdx.x] = 0xffffffffu;
  else if (threadIdx.x < 6) sb[threadIdx.x] = 0u;
  if (threadIdx.x == 0) scount = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    float mu[3], ls[3], q[4];
    for (int k = 0; k < 3; k++) { mu[k] = means[3 * i + k]; ls[k] = log_scales[3 * i + k]; }
    for (int k = 0; k < 4; k++) q[k] = quats[4 * i + k];
    const float sig = density[i];
    const float qn2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    bool ok = isfinite(mu[0]) && isfinite(mu[1]) && isfinite(mu[2]) && isfinite(ls[0]) &&
              isfinite(ls[1]) && isfinite(ls[2]) && isfinite(qn2) && qn2 > 0.0f &&
              isfinite(sig) && sig > sigma_eps;
    float s[3];
    for (int k = 0; k < 3; k++) { s[k] = expf(ls[k]); ok = ok && s[k] > 0.0f && isfinite(s[k]); }
    float g[kGeomFloats];
    for (int k = 0; k < kGeomFloats; k++) g[k] = 0.0f;
    float lo[3] = {1.0f, 1.0f, 1.0f}, hi[3] = {-1.0f, -1.0f, -1.0f};
    float ax[kAuxFloats] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (ok) {
      const float rn = rsqrtf(qn2);
      ax[0] = s[0]; ax[1] = s[1]; ax[2] = s[2];
      ax[7] = sqrtf(qn2);
      ax[3] = q[0] / ax[7]; ax[4] = q[1] / ax[7]; ax[5] = q[2] / ax[7]; ax[6] = q[3] / ax[7];
      const float w = q[0] * rn, x = q[1] * rn, y = q[2] * rn, z = q[3] * rn;
      float R[9];
      R[0] = 1.0f - 2.0f * (y * y + z * z); R[1] = 2.0f * (x * y - w * z); R[2] = 2.0f * (x * z + w * y);
      R[3] = 2.0f * (x * y + w * z); R[4] = 1.0f - 2.0f * (x * x + z * z); R[5] = 2.0f * (y * z - w * x);
      R[6] = 2.0f * (x * z - w * y); R[7] = 2.0f * (y * z + w * x); R[8] = 1.0f - 2.0f * (x * x + y * y);
      const float k2 = 2.0f * logf(sig / sigma_eps);
      const float k = sqrtf(k2);
      for (int r = 0; r < 3; r++) {
        g[G_MU + r] = mu[r];
        // row r of M = S^-1 R^T is column r of R divided by s_r
        for (int c = 0; c < 3; c++) g[G_M + 3 * r + c] = R[3 * c + r] / s[r];
      }
      g[G_K2] = k2;
      g[G_SIG] = sig;
      g[G_L2SIG] = log2f(sig);
      // minimal AABB half-lengths L_i = k sqrt(sum_j r_ij^2 s_j^2) (Supp. B), padded
      // outward so that every point of an FP32 ray/ellipsoid interval lies inside
      float amax = fmaxf(fabsf(mu[0]), fmaxf(fabsf(mu[1]), fabsf(mu[2])));
      for (int r = 0; r < 3; r++) {
        float acc = 0.0f;
        for (int c = 0; c < 3; c++) acc += R[3 * r + c] * R[3 * r + c] * s[c] * s[c];
        float L = k * sqrtf(acc);
        L = L * 1.0001f + 2e-6f * (amax + L) + 1e-30f;
        lo[r] = mu[r] - L;
        hi[r] = mu[r] + L;
      }
      // bounding sphere of the ellipsoid: radius k max(s), padded like L
      float rad = k * fmaxf(s[0], fmaxf(s[1], s[2]));
      g[G_RAD] = rad * 1.0001f + 2e-6f * (amax + rad) + 1e-30f;
      atomicMin(&sb[0], f2ord(mu[0])); atomicMin(&sb[1], f2ord(mu[1])); atomicMin(&sb[2], f2ord(mu[2]));
      atomicMax(&sb[3], f2ord(mu[0])); atomicMax(&sb[4], f2ord(mu[1])); atomicMax(&sb[5], f2ord(mu[2]));
      atomicAdd(&scount, 1);
    }
    float4 *gp = reinterpret_cast<float4 *>(geom + (size_t)kGeomFloats * i);
    for (int k = 0; k < 4; k++) gp[k] = make_float4(g[4 * k], g[4 * k + 1], g[4 * k + 2], g[4 * k + 3]);
    for (int k = 0; k < 3; k++) { aabb[6 * i + k] = lo[k]; aabb[6 * i + 3 + k] = hi[k]; }
    for (int k = 0; k < kAuxFloats; k++) aux[kAuxFloats * i + k] = ax[k];
    active[i] = ok ? 1 : 0;
  }
  __syncthreads();
  if (threadIdx.x < 3) atomicMin(&bounds[threadIdx.x], sb[threadIdx.x]);
  else if (threadIdx.x < 6) atomicMax(&bounds[threadIdx.x], sb[threadIdx.x]);
  if (threadIdx.x == 0 && scount) atomicAdd(&counters[0], scount);
}

// Spherical-Gaussian lobes (user order): lobe j of the user record (amplitude
// rgb, axis xyz, sharpness) becomes (amplitude rgb, sharpness, unit axis,
// |xi|); absent lobes (j >= n_sg, a zero or non-finite axis) are all zero, so
// they add nothing to the colour and get no gradient.
__global__ __launch_bounds__(256) void k_sg_pack(int64_t n, int n_sg, const float *__restrict__ sg,
                                                 float *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int j = 0; j < kMaxSg; j++) {
    float r[kSgLobeFloats] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (j < n_sg) {
      const float *p = sg + ((size_t)i * n_sg + j) * kSgUserFloats;
      const float xn = sqrtf(p[3] * p[3] + p[4] * p[4] + p[5] * p[5]);
      if (xn > 0.0f && isfinite(xn)) {
        r[0] = p[0]; r[1] = p[1]; r[2] = p[2];
        r[3] = p[6];
        r[4] = p[3] / xn; r[5] = p[4] / xn; r[6] = p[5] / xn;
        r[7] = xn;
      }
    }
    float4 *o = reinterpret_cast<float4 *>(out + (size_t)kSgFloats * i + kSgLobeFloats * j);
    o[0] = make_float4(r[0], r[1], r[2], r[3]);
    o[1] = make_float4(r[4], r[5], r[6], r[7]);
  }
}

// Spread the low 21 bits of v so that bit b lands at bit 3b.
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

// Z-order index of the normalised, quantised mean (Sec. 3.3).  Inactive
// Gaussians get the key 2^(3*bits), above every active key.
__global__ __launch_bounds__(256) void k_morton(int64_t n, const float *__restrict__ means,
                                                const uint8_t *__restrict__ active,
                                                const uint32_t *__restrict__ bounds, int bits,
                                                uint64_t *__restrict__ keys,
                                                uint32_t *__restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t key = 1ull << (3 * bits);
  if (active[i]) {
    const float qmax = (float)((1u << bits) - 1u);
    uint64_t c[3];
    for (int k = 0; k < 3; k++) {
      const float lo = ord2f(bounds[k]), hi = ord2f(bounds[3 + k]);
      const float ext = hi - lo;
      float u = ext > 0.0f ? (means[3 * i + k] - lo) / ext : 0.0f;
      u = fminf(fmaxf(u, 0.0f), 1.0f);
      c[k] = (uint64_t)(u * qmax + 0.5f);
      if (c[k] > (uint64_t)qmax) c[k] = (uint64_t)qmax;
    }
    key = (spread3(c[0]) << 2) | (spread3(c[1]) << 1) | spread3(c[2]);
  }
  keys[i] = key;
  vals[i] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort, 8-bit digits.  Each block owns a tile of
// kSortItems keys; a pass is histogram -> global exclusive scan (digit-major)
// -> stable scatter with per-wave ballot multisplit.

constexpr int kSortThreads = 256;
constexpr int kSortRounds = 16;
constexpr int kSortItems = kSortThreads * kSortRounds;

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint64_t *__restrict__ keys,
                                                             int64_t n, int shift,
                                                             uint32_t *__restrict__ hist,
                                                             int nblocks) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortItems;
  for (int r = 0; r < kSortRounds; r++) {
    const int64_t i = base + r * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 0xff], 1u);
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of `count` uint32 in place; a single block of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan_exclusive(uint32_t *__restrict__ data, int64_t count) {
  __shared__ uint32_t wsum[16];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int64_t base = 0; base < count; base += 1024) {
    const int64_t i = base + threadIdx.x;
    uint32_t v = i < count ? data[i] : 0u;
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
      uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    if (wid == 0) {
      uint32_t s = lane < 16 ? wsum[lane] : 0u;
      for (int o = 1; o < 16; o <<= 1) {
        uint32_t y = __shfl_up(s, o, 64);
        if (lane >= o) s += y;
      }
      if (lane < 16) wsum[lane] = s;
    }
    __syncthreads();
    const uint32_t before = carry + (wid ? wsum[wid - 1] : 0u) + x - v;
    if (i < count) data[i] = before;
    __syncthreads();
    if (threadIdx.x == 1023) carry = before + v;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint64_t *__restrict__ keys_in, const uint32_t *__restrict__ vals_in,
    uint64_t *__restrict__ keys_out, uint32_t *__restrict__ vals_out, int64_t n, int shift,
    const uint32_t *__restrict__ hist, int nblocks) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcount[kWavesPerBlock][256];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  base[threadIdx.x] = hist[(size_t)threadIdx.x * nblocks + blockIdx.x];
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t tile = (int64_t)blockIdx.x * kSortItems;
  for (int r = 0; r < kSortRounds; r++) {
    for (int w = 0; w < kWavesPerBlock; w++) wcount[w][threadIdx.x] = 0;
    __syncthreads();
    const int64_t i = tile + r * kSortThreads + threadIdx.x;
    const bool valid = i < n;
    uint64_t key = 0;
    uint32_t val = 0;
    uint32_t digit = 0;
    if (valid) { key = keys_in[i]; val = vals_in[i]; digit = (uint32_t)(key >> shift) & 0xffu; }
    // lanes of this wave holding the same digit
    uint64_t same = ballot(valid);
    for (int b = 0; b < 8; b++) {
      const uint64_t bal = ballot(((digit >> b) & 1u) != 0);
      same &= ((digit >> b) & 1u) ? bal : ~bal;
    }
    const uint32_t rank = (uint32_t)__popcll(same & lt_mask);
    if (valid && rank == 0) wcount[wid][digit] = (uint32_t)__popcll(same);
    __syncthreads();
    if (valid) {
      uint32_t off = base[digit] + rank;
      for (int w = 0; w < wid; w++) off += wcount[w][digit];
      keys_out[off] = key;
      vals_out[off] = val;
    }
    __syncthreads();
    uint32_t tot = 0;
    for (int w = 0; w < kWavesPerBlock; w++) tot += wcount[w][threadIdx.x];
    base[threadIdx.x] += tot;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Z-ordered pack of the geometry, colour and AABB records of active Gaussians.
// Z-ordered pack, one array at a time: dst row i = src row perm[i] (its
// first src_cols floats, zero padding up to dst_stride).  One thread per
// destination float, so the reads of a source row are contiguous and each
// record's cache lines are fetched once.
__global__ __launch_bounds__(256) void k_gather_rows(int64_t n, const int32_t *__restrict__ counters,
                                                     const uint32_t *__restrict__ perm,
                                                     const float *__restrict__ src, int src_stride,
                                                     int src_cols, float *__restrict__ dst,
                                                     int dst_stride) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = f / dst_stride;
  const int k = (int)(f - i * dst_stride);
  if (i >= n || i >= counters[0]) return;
  dst[f] = k < src_cols ? src[(size_t)perm[i] * src_stride + k] : 0.0f;
}

// Node boxes without inter-thread synchronisation: a segment tree (heap
// layout, P leaves, P a power of two) over the Z-ordered leaf boxes gives the
// union of any leaf range in O(log P) reads; every internal node's child
// boxes are the unions of its two child ranges.
__global__ __launch_bounds__(256) void k_seg_leaves(int64_t P, const int32_t *__restrict__ counters,
                                                    const float *__restrict__ aabb,
                                                    float *__restrict__ seg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const int n = counters[0];
  float *d = seg + 6 * (size_t)(P + i);
  if (i < n) {
    for (int k = 0; k < 6; k++) d[k] = aabb[6 * i + k];
  } else {
    for (int k = 0; k < 3; k++) { d[k] = __builtin_huge_valf(); d[3 + k] = -__builtin_huge_valf(); }
  }
}

__global__ __launch_bounds__(256) void k_seg_level(int64_t lo, int64_t hi, float *__restrict__ seg) {
  const int64_t k = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= hi) return;
  const float *a = seg + 6 * (size_t)(2 * k), *b = seg + 6 * (size_t)(2 * k + 1);
  float *d = seg + 6 * (size_t)k;
  for (int c = 0; c < 3; c++) { d[c] = fminf(a[c], b[c]); d[3 + c] = fmaxf(a[3 + c], b[3 + c]); }
}

// Union of the boxes of leaves [l, r] (inclusive).
__device__ __forceinline__ void seg_query(const float *__restrict__ seg, int64_t P, int64_t l,
                                          int64_t r, float *box) {
  for (int c = 0; c < 3; c++) { box[c] = __builtin_huge_valf(); box[3 + c] = -__builtin_huge_valf(); }
  l += P;
  r += P + 1;
  while (l < r) {
    if (l & 1) {
      const float *x = seg + 6 * (size_t)l++;
      for (int c = 0; c < 3; c++) { box[c] = fminf(box[c], x[c]); box[3 + c] = fmaxf(box[3 + c], x[3 + c]); }
    }
    if (r & 1) {
      const float *x = seg + 6 * (size_t)(--r);
      for (int c = 0; c < 3; c++) { box[c] = fminf(box[c], x[c]); box[3 + c] = fmaxf(box[3 + c], x[3 + c]); }
    }
    l >>= 1;
    r >>= 1;
  }
}

// ---------------------------------------------------------------------------
// Karras LBVH over the sorted keys of the active Gaussians.  Internal node i
// covers a key range with i at one end; duplicate keys are split by index.
__device__ __forceinline__ int lcp(const uint64_t *__restrict__ k, int n, int i, int j) {
  if (j < 0 || j >= n) return -1;
  const uint64_t a = k[i], b = k[j];
  if (a == b) return 64 + __clz((uint32_t)(i ^ j));
  return __clzll(a ^ b);
}

__global__ __launch_bounds__(256) void k_lbvh_hierarchy(int64_t n_max,
                                                        const int32_t *__restrict__ counters,
                                                        const uint64_t *__restrict__ keys,
                                                        const float *__restrict__ aabb,
                                                        const float *__restrict__ seg, int64_t P,
                                                        float4 *__restrict__ nodes) {
  const int n = counters[0];
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= n_max) return;
  const int i = (int)tid;
  if (n == 1 && i == 0) {
    nodes[0] = make_float4(aabb[0], aabb[1], aabb[2], __int_as_float(~0));
    nodes[1] = make_float4(aabb[3], aabb[4], aabb[5], __int_as_float(kNoChild));
    nodes[2] = make_float4(0.f, 0.f, 0.f, __int_as_float(0));
    nodes[3] = make_float4(0.f, 0.f, 0.f, __int_as_float(0));
    return;
  }
  if (i >= n - 1) return;
  const int d = (lcp(keys, n, i, i + 1) - lcp(keys, n, i, i - 1)) >= 0 ? 1 : -1;
  const int dmin = lcp(keys, n, i, i - d);
  int64_t lmax = 2;
  while (lmax < 2 * (int64_t)n && lcp(keys, n, i, (int)(i + lmax * d)) > dmin) lmax <<= 1;
  int l = 0;
  for (int64_t t = lmax >> 1; t >= 1; t >>= 1) {
    const int64_t jj = i + (l + t) * d;
    if (jj >= 0 && jj < n && lcp(keys, n, i, (int)jj) > dmin) l += (int)t;
  }
  const int j = i + l * d;
  const int dnode = lcp(keys, n, i, j);
  int s = 0;
  int t = l;
  do {
    t = (t + 1) >> 1;
    if (lcp(keys, n, i, i + (s + t) * d) > dnode) s += t;
  } while (t > 1);
  const int gamma = i + s * d + (d < 0 ? -1 : 0);
  const int lo = i < j ? i : j, hi = i < j ? j : i;
  const int left = (lo == gamma) ? ~gamma : gamma;
  const int right = (hi == gamma + 1) ? ~(gamma + 1) : gamma + 1;
  float bl[6], br[6];
  seg_query(seg, P, lo, gamma, bl);
  seg_query(seg, P, gamma + 1, hi, br);
  float4 *nd = nodes + 4 * (size_t)i;
  nd[0] = make_float4(bl[0], bl[1], bl[2], __int_as_float(left));
  nd[1] = make_float4(bl[3], bl[4], bl[5], __int_as_float(right));
  // the node's leaf (Z index) range [lo, hi]; the split is implied by the
  // left link (gamma), so range-restricted traversals can prune children
  nd[2] = make_float4(br[0], br[1], br[2], __int_as_float(lo));
  nd[3] = make_float4(br[3], br[4], br[5], __int_as_float(hi));
}

// 4-wide nodes by surface-area collapse: every binary internal node gathers
// its two children and then, while it has fewer than four, replaces the
// internal child of largest box surface area by that child's two children
// (in place, so the record stays in left-to-right Z order).  Every internal
// node gets a record, indexed by its binary index, so a link to an internal
// child is that child's binary index.
__global__ __launch_bounds__(256) void k_bvh4(int64_t n_max, const int32_t *__restrict__ counters,
                                              const float4 *__restrict__ nodes,
                                              float *__restrict__ nodes4) {
  const int n = counters[0];
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int n_inner = n > 1 ? n - 1 : 1;
  if (tid >= n_max || n <= 0 || tid >= n_inner) return;
  const int i = (int)tid;
  int lk[4];
  float4 blo[4], bhi[4];
  int m = 0;
  {
    const float4 a = nodes[4 * (size_t)i], b = nodes[4 * (size_t)i + 1], c = nodes[4 * (size_t)i + 2],
                 d = nodes[4 * (size_t)i + 3];
    const int l0 = __float_as_int(a.w), l1 = __float_as_int(b.w);
    if (l0 != kNoChild) { lk[m] = l0; blo[m] = a; bhi[m] = b; m++; }
    if (l1 != kNoChild) { lk[m] = l1; blo[m] = c; bhi[m] = d; m++; }
  }
  while (m < 4) {
    int best = -1;
    float bsa = -1.0f;
    for (int k = 0; k < m; k++) {
      if (lk[k] < 0 || lk[k] >= n_inner) continue;
      const float dx = bhi[k].x - blo[k].x, dy = bhi[k].y - blo[k].y, dz = bhi[k].z - blo[k].z;
      const float sa = dx * dy + dy * dz + dz * dx;
      if (sa > bsa) { bsa = sa; best = k; }
    }
    if (best < 0) break;
    const int x = lk[best];
    const float4 a = nodes[4 * (size_t)x], b = nodes[4 * (size_t)x + 1], c = nodes[4 * (size_t)x + 2],
                 d = nodes[4 * (size_t)x + 3];
    const int l0 = __float_as_int(a.w), l1 = __float_as_int(b.w);
    if (l0 == kNoChild || l1 == kNoChild) break;   // only the root of a one-leaf tree has one child
    for (int k = m; k > best + 1; k--) { lk[k] = lk[k - 1]; blo[k] = blo[k - 1]; bhi[k] = bhi[k - 1]; }
    lk[best] = l0; blo[best] = a; bhi[best] = b;
    lk[best + 1] = l1; blo[best + 1] = c; bhi[best + 1] = d;
    m++;
  }
  float f[kNode4Floats];
  for (int k = 0; k < 24; k++) f[k] = 0.0f;
  for (int k = 0; k < 4; k++) {
    f[24 + k] = __int_as_float(kNoChild);
    f[28 + 2 * k] = __int_as_float(1);        // empty range
    f[29 + 2 * k] = __int_as_float(0);
  }
  for (int k = 0; k < m; k++) {
    f[6 * k + 0] = blo[k].x; f[6 * k + 1] = blo[k].y; f[6 * k + 2] = blo[k].z;
    f[6 * k + 3] = bhi[k].x; f[6 * k + 4] = bhi[k].y; f[6 * k + 5] = bhi[k].z;
    f[24 + k] = __int_as_float(lk[k]);
    int first = ~lk[k], last = ~lk[k];
    if (lk[k] >= 0) {
      first = __float_as_int(nodes[4 * (size_t)lk[k] + 2].w);
      last = __float_as_int(nodes[4 * (size_t)lk[k] + 3].w);
    }
    f[28 + 2 * k] = __int_as_float(first);
    f[29 + 2 * k] = __int_as_float(last);
  }
  float4 *out = reinterpret_cast<float4 *>(nodes4 + (size_t)kNode4Floats * i);
  for (int k = 0; k < kNode4Floats / 4; k++)
    out[k] = make_float4(f[4 * k], f[4 * k + 1], f[4 * k + 2], f[4 * k + 3]);
}

// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_build(const BuildArgs &a, hipStream_t st) {
  const int64_t n = a.n;
  k_build_init<<<1, 64, 0, st>>>(a.bounds, a.counters);
  k_preprocess<<<nblk(n, 256), 256, 0, st>>>(n, a.means, a.log_scales, a.quats, a.density,
                                             a.sigma_eps, a.geom_user, a.aabb_user, a.aux_user, a.active,
                                             a.bounds, a.counters);
  k_morton<<<nblk(n, 256), 256, 0, st>>>(n, a.means, a.active, a.bounds, a.morton_bits,
                                         a.keys[0], a.vals[0]);
  const int nb = (int)nblk(n, kSortItems);
  const int passes = (3 * a.morton_bits + 1 + 7) / 8;
  int cur = 0;
  for (int p = 0; p < passes; p++) {
    const int shift = 8 * p;
    k_radix_hist<<<nb, kSortThreads, 0, st>>>(a.keys[cur], n, shift, a.sort_hist, nb);
    k_scan_exclusive<<<1, 1024, 0, st>>>(a.sort_hist, (int64_t)256 * nb);
    k_radix_scatter<<<nb, kSortThreads, 0, st>>>(a.keys[cur], a.vals[cur], a.keys[cur ^ 1],
                                                 a.vals[cur ^ 1], n, shift, a.sort_hist, nb);
    cur ^= 1;
  }
  *a.sorted_sel = cur;
  const uint32_t *perm = a.vals[cur];
  k_gather_rows<<<nblk(n * kGeomFloats, 256), 256, 0, st>>>(n, a.counters, perm, a.geom_user,
                                                            kGeomFloats, kGeomFloats, a.geom,
                                                            kGeomFloats);
  k_gather_rows<<<nblk(n * 6, 256), 256, 0, st>>>(n, a.counters, perm, a.aabb_user, 6, 6, a.aabb, 6);
  k_gather_rows<<<nblk(n * kAuxFloats, 256), 256, 0, st>>>(n, a.counters, perm, a.aux_user,
                                                           kAuxFloats, kAuxFloats, a.aux,
                                                           kAuxFloats);
  k_gather_rows<<<nblk(n * a.col_stride, 256), 256, 0, st>>>(n, a.counters, perm, a.sh,
                                                             3 * a.sh_k, 3 * a.sh_k, a.col,
                                                             a.col_stride);
  if (a.n_sg > 0) {
    k_sg_pack<<<nblk(n, 256), 256, 0, st>>>(n, a.n_sg, a.sg, a.sg_user);
    k_gather_rows<<<nblk(n * kSgFloats, 256), 256, 0, st>>>(n, a.counters, perm, a.sg_user,
                                                           kSgFloats, kSgFloats, a.sgrec, kSgFloats);
  }
  int64_t P = 1;
  while (P < n) P <<= 1;
  k_seg_leaves<<<nblk(P, 256), 256, 0, st>>>(P, a.counters, a.aabb, a.seg);
  for (int64_t lo = P >> 1; lo >= 1; lo >>= 1)
    k_seg_level<<<nblk(lo, 256), 256, 0, st>>>(lo, 2 * lo, a.seg);
  k_lbvh_hierarchy<<<nblk(n, 256), 256, 0, st>>>(n, a.counters, a.keys[cur], a.aabb, a.seg, P,
                                                 reinterpret_cast<float4 *>(a.nodes));
  k_bvh4<<<nblk(n, 256), 256, 0, st>>>(n, a.counters, reinterpret_cast<const float4 *>(a.nodes),
                                       a.nodes4);
  return hipGetLastError();
}

}  // namespace rgx

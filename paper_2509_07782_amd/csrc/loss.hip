// Isotropic scale loss (Sec. 3.4, Eq. 8 with the AABB/ellipsoid volume-ratio
// bound of Eq. 7 and Eq. 9).  For a Gaussian with scales s = exp(l) the bound
// is r = 2 / (pi sqrt 3) * (sum_j s_j^2)^(3/2) / prod_j s_j, and the loss is
// the mean over the n Gaussians of max(r, r0) - r0.  Its gradient follows
// from ln r = const + 3/2 ln(sum s^2) - sum l:
//   d r / d l_j = r (3 s_j^2 / sum s^2 - 1),
//   dL / d l_j = [r > r0] (d r / d l_j) / n.
// The sum is reduced deterministically: fixed per-block partial sums in a
// first launch, a single block adding them in a fixed order in a second.
#include "common.hpp"
#include "internal.hpp"

namespace rgx {

constexpr int kLossThreads = 256;

__global__ __launch_bounds__(kLossThreads) void k_iso_partial(int64_t n, const float *__restrict__ ls,
                                                              float r0, float inv_n,
                                                              float *__restrict__ grad,
                                                              int accumulate,
                                                              double *__restrict__ partial) {
  __shared__ double red[kLossThreads];
  const int64_t i = (int64_t)blockIdx.x * kLossThreads + threadIdx.x;
  double term = 0.0;
  if (i < n) {
    const float s0 = expf(ls[3 * i]), s1 = expf(ls[3 * i + 1]), s2 = expf(ls[3 * i + 2]);
    const float q0 = s0 * s0, q1 = s1 * s1, q2 = s2 * s2;
    const float sum = q0 + q1 + q2;
    // (sum s^2)^(3/2) / prod s, formed in logs to stay in range
    const float lr = 1.5f * logf(sum) - (ls[3 * i] + ls[3 * i + 1] + ls[3 * i + 2]);
    const float r = 0.36755259694786136f * expf(fminf(lr, 80.0f));   // 2 / (pi sqrt 3)
    const bool over = r > r0;
    term = over ? (double)r - (double)r0 : 0.0;
    const float g = over ? r * inv_n : 0.0f;
    const float inv = 1.0f / sum;
    const float d0 = g * (3.0f * q0 * inv - 1.0f), d1 = g * (3.0f * q1 * inv - 1.0f),
                d2 = g * (3.0f * q2 * inv - 1.0f);
    if (accumulate) {
      grad[3 * i] += d0; grad[3 * i + 1] += d1; grad[3 * i + 2] += d2;
    } else {
      grad[3 * i] = d0; grad[3 * i + 1] = d1; grad[3 * i + 2] = d2;
    }
  }
  red[threadIdx.x] = term;
  __syncthreads();
  for (int h = kLossThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kLossThreads) void k_iso_final(int64_t nb, const double *__restrict__ partial,
                                                            double inv_n, float *__restrict__ loss) {
  __shared__ double red[kLossThreads];
  double acc = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += kLossThreads) acc += partial[b];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kLossThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)(red[0] * inv_n);
}

int64_t iso_blocks(int64_t n) { return (n + kLossThreads - 1) / kLossThreads; }

// Fixed workspace of the allocation-free entry point: one partial sum per
// block for the largest supported n (256 KB per device, held until the
// process ends).  Host code never passes the array's name to a kernel; it
// uses the device address resolved once per device by iso_scratch_resolve.
constexpr int64_t kIsoScratchDoubles = (RGX_MAX_GAUSSIANS_INTERNAL + kLossThreads - 1) / kLossThreads;
static __device__ __align__(256) double scratch[kIsoScratchDoubles];

int64_t iso_scratch_capacity() { return kIsoScratchDoubles; }

hipError_t iso_scratch_resolve(double **ptr) {
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  *ptr = e == hipSuccess ? (double *)p : nullptr;
  return e;
}

hipError_t launch_isotropic_loss(int64_t n, const float *log_scales, float r0, float *loss,
                                 float *grad, int accumulate, double *partial, hipStream_t st) {
  const int64_t nb = iso_blocks(n);
  k_iso_partial<<<(unsigned)nb, kLossThreads, 0, st>>>(n, log_scales, r0, (float)(1.0 / (double)n),
                                                       grad, accumulate, partial);
  k_iso_final<<<1, kLossThreads, 0, st>>>(nb, partial, 1.0 / (double)n, loss);
  return hipGetLastError();
}

}  // namespace rgx

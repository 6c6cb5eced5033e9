// Adam (Kingma and Ba, 2015) for the training workload: one step over
// several parameter arrays.  The step counter lives in device memory and is
// advanced by a kernel, so a graph that captured the step replays with the
// right bias corrections.  Elementwise, coalesced, grid-stride.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace rgx {

__global__ void k_adam_tick(int32_t *step) { *step += 1; }

__global__ __launch_bounds__(256) void k_adam(int64_t n, float *__restrict__ p,
                                              const float *__restrict__ g, float *__restrict__ m,
                                              float *__restrict__ v, float lr, float b1, float b2,
                                              float eps, const int32_t *__restrict__ step) {
  const float t = (float)*step;
  // bias corrections 1 / (1 - b^t)
  const float c1 = 1.0f / (1.0f - powf(b1, t));
  const float c2 = 1.0f / (1.0f - powf(b2, t));
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float gi = g[i];
    const float mi = fmaf(b1, m[i], (1.0f - b1) * gi);
    const float vi = fmaf(b2, v[i], (1.0f - b2) * (gi * gi));
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  }
}

hipError_t launch_adam_tick(int32_t *step, hipStream_t st) {
  k_adam_tick<<<1, 1, 0, st>>>(step);
  return hipGetLastError();
}

hipError_t launch_adam(int64_t n, float *p, const float *g, float *m, float *v, float lr, float b1,
                       float b2, float eps, const int32_t *step, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t nb = (n + 255) / 256;
  if (nb > 8192) nb = 8192;
  k_adam<<<(unsigned)nb, 256, 0, st>>>(n, p, g, m, v, lr, b1, b2, eps, step);
  return hipGetLastError();
}

}  // namespace rgx

// Adam update of the design phases (the optimiser of the differentiable
// form's design loop): one elementwise pass over phi, its gradient and the two
// moment estimates, stream-ordered, with the step number read from device
// memory so that the whole design step can be captured in a graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>

#include "gswmtp_internal.h"

namespace {

// Kingma and Ba's update with bias-corrected moments, in float32:
//   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
//   phi -= (lr / (1 - b1^t)) m / (sqrt(v) / sqrt(1 - b2^t) + eps).
__global__ __launch_bounds__(256) void k_adam(float *phi, const float *grad, float *m, float *v,
                                              const float *step, size_t n, float lr, float b1,
                                              float b2, float eps) {
  const float t = *step;
  const float bc1 = 1.f - powf(b1, t), bc2 = 1.f - powf(b2, t);
  const float step_size = lr / bc1, rbc2 = 1.f / sqrtf(bc2);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    phi[i] -= step_size * mi / (sqrtf(vi) * rbc2 + eps);
  }
}

}  // namespace

extern "C" int gswmtp_adam_step_device(float *phi, const float *grad, float *m, float *v,
                                       const float *step, size_t n, double lr, double beta1,
                                       double beta2, double eps, void *stream) {
  if (n == 0) return GSWMTP_OK;
  if (!phi || !grad || !m || !v || !step) return GSWMTP_E_INVAL;
  if (!std::isfinite(lr) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
      !(eps >= 0.0) || !std::isfinite(eps))
    return GSWMTP_E_INVAL;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0,
                     static_cast<hipStream_t>(stream), phi, grad, m, v, step, n, (float)lr,
                     (float)beta1, (float)beta2, (float)eps);
  return hipGetLastError() == hipSuccess ? GSWMTP_OK : GSWMTP_E_HIP;
}

// The differentiable form's design loop on the device: the design loss of
// the foci intensities with its gradient, and the Adam update of the phases.
// Both are stream-ordered and read everything they need from device memory,
// so that a whole design step can be captured in a graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>

#include "adam_update.h"
#include "gswmtp_internal.h"

namespace {

using gswmtp::adam_apply;
using gswmtp::adam_scalars;

// Kingma and Ba's update with bias-corrected moments (adam_update.h), one
// value per thread.
__global__ __launch_bounds__(256) void k_adam(float *phi, const float *grad, float *m, float *v,
                                              const float *step, size_t n, float lr, float b1,
                                              float b2, float eps) {
  float step_size, rbc2;
  adam_scalars(*step, lr, b1, b2, step_size, rbc2);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    float mi = m[i], vi = v[i], p = phi[i];
    adam_apply(p, mi, vi, grad[i], b1, b2, step_size, rbc2, eps);
    m[i] = mi;
    v[i] = vi;
    phi[i] = p;
  }
}

// The same update, four values per thread with 16-byte accesses (n a
// multiple of 4, every pointer 16-byte aligned).
__global__ __launch_bounds__(256) void k_adam4(float4 *phi, const float4 *grad, float4 *m,
                                               float4 *v, const float *step, size_t n4,
                                               float lr, float b1, float b2, float eps) {
  float step_size, rbc2;
  adam_scalars(*step, lr, b1, b2, step_size, rbc2);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
       i += (size_t)gridDim.x * blockDim.x) {
    const float4 g = grad[i];
    float4 mi = m[i], vi = v[i], p = phi[i];
    adam_apply(p.x, mi.x, vi.x, g.x, b1, b2, step_size, rbc2, eps);
    adam_apply(p.y, mi.y, vi.y, g.y, b1, b2, step_size, rbc2, eps);
    adam_apply(p.z, mi.z, vi.z, g.z, b1, b2, step_size, rbc2, eps);
    adam_apply(p.w, mi.w, vi.w, g.w, b1, b2, step_size, rbc2, eps);
    m[i] = mi;
    v[i] = vi;
    phi[i] = p;
  }
}

// Design loss L = sum_n (i_n - t_n)^2 - w eta and dL/dI, one workgroup:
// i = I / sum I, t = T / sum T, eta = sum I / (n_ap sum A^2).  Sums in
// float64 over a fixed tree (strided per thread, then a shared-memory tree),
// so the result is the same on every run.
constexpr int kLossThreads = 1024;

__device__ __forceinline__ double block_sum(double x, double *sh) {
  const int t = threadIdx.x;
  sh[t] = x;
  __syncthreads();
  for (int w = kLossThreads / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// With `step` (the design loop's bookkeeping, optional): thread 0 also
// writes L to hist[*step] (while *step < hist_cap) and advances *step by one,
// the step number that the Adam update launched after it reads.
__global__ __launch_bounds__(kLossThreads) void k_design_loss(const float *I, const float *T,
                                                              int n, double c, double w,
                                                              float *loss, float *dI,
                                                              float *hist, int hist_cap,
                                                              float *step) {
  __shared__ double sh[kLossThreads];
  double sI = 0.0, sT = 0.0;
  for (int k = threadIdx.x; k < n; k += kLossThreads) {
    sI += (double)I[k];
    sT += (double)T[k];
  }
  const double SI = block_sum(sI, sh), ST = block_sum(sT, sh);
  double rr = 0.0, ri = 0.0;
  for (int k = threadIdx.x; k < n; k += kLossThreads) {
    const double i = (double)I[k] / SI, r = i - (double)T[k] / ST;
    rr += r * r;
    ri += r * i;
  }
  const double RR = block_sum(rr, sh), RI = block_sum(ri, sh);
  if (threadIdx.x == 0) {
    const float L = (float)(RR - w * SI * c);
    *loss = L;
    if (step) {
      const float s = *step;
      if (hist && s >= 0.f && s < (float)hist_cap) hist[(int)s] = L;
      *step = s + 1.f;
    }
  }
  // d i_m / d I_k = (delta_mk - i_m) / S
  for (int k = threadIdx.x; k < n; k += kLossThreads) {
    const double r = (double)I[k] / SI - (double)T[k] / ST;
    dI[k] = (float)(2.0 * r / SI - 2.0 * RI / SI - w * c);
  }
}

}  // namespace

namespace {

int design_loss(const float *dev_I, const float *dev_target, int n, double n_ap, double sum_a2,
                double eta_weight, float *dev_loss, float *dev_dI, float *dev_hist,
                int hist_cap, float *dev_step, void *stream) {
  if (n < 1 || !dev_I || !dev_target || !dev_loss || !dev_dI) return GSWMTP_E_INVAL;
  if (!(n_ap > 0.0) || !(sum_a2 > 0.0) || !std::isfinite(n_ap) || !std::isfinite(sum_a2) ||
      !std::isfinite(eta_weight))
    return GSWMTP_E_INVAL;
  hipLaunchKernelGGL(k_design_loss, dim3(1), dim3(kLossThreads), 0,
                     static_cast<hipStream_t>(stream), dev_I, dev_target, n,
                     1.0 / (n_ap * sum_a2), eta_weight, dev_loss, dev_dI, dev_hist, hist_cap,
                     dev_step);
  return hipGetLastError() == hipSuccess ? GSWMTP_OK : GSWMTP_E_HIP;
}

}  // namespace

extern "C" int gswmtp_design_loss_device(const float *dev_I, const float *dev_target, int n,
                                         double n_ap, double sum_a2, double eta_weight,
                                         float *dev_loss, float *dev_dI, void *stream) {
  return design_loss(dev_I, dev_target, n, n_ap, sum_a2, eta_weight, dev_loss, dev_dI, nullptr,
                     0, nullptr, stream);
}

extern "C" int gswmtp_design_loss_record_device(const float *dev_I, const float *dev_target,
                                                int n, double n_ap, double sum_a2,
                                                double eta_weight, float *dev_loss,
                                                float *dev_dI, float *dev_hist, int hist_cap,
                                                float *dev_step, void *stream) {
  if (!dev_step || hist_cap < 0 || (hist_cap > 0 && !dev_hist)) return GSWMTP_E_INVAL;
  return design_loss(dev_I, dev_target, n, n_ap, sum_a2, eta_weight, dev_loss, dev_dI, dev_hist,
                     hist_cap, dev_step, stream);
}

extern "C" int gswmtp_adam_step_device(float *phi, const float *grad, float *m, float *v,
                                       const float *step, size_t n, double lr, double beta1,
                                       double beta2, double eps, void *stream) {
  if (n == 0) return GSWMTP_OK;
  if (!phi || !grad || !m || !v || !step) return GSWMTP_E_INVAL;
  if (!std::isfinite(lr) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
      !(eps >= 0.0) || !std::isfinite(eps))
    return GSWMTP_E_INVAL;
  const auto aligned = [](const void *q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
  if (n % 4 == 0 && aligned(phi) && aligned(grad) && aligned(m) && aligned(v)) {
    const size_t n4 = n / 4, blocks = std::min<size_t>((n4 + 255) / 256, 8192);
    hipLaunchKernelGGL(k_adam4, dim3((unsigned)blocks), dim3(256), 0,
                       static_cast<hipStream_t>(stream), reinterpret_cast<float4 *>(phi),
                       reinterpret_cast<const float4 *>(grad), reinterpret_cast<float4 *>(m),
                       reinterpret_cast<float4 *>(v), step, n4, (float)lr, (float)beta1,
                       (float)beta2, (float)eps);
  } else {
    const size_t blocks = std::min<size_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0,
                       static_cast<hipStream_t>(stream), phi, grad, m, v, step, n, (float)lr,
                       (float)beta1, (float)beta2, (float)eps);
  }
  return hipGetLastError() == hipSuccess ? GSWMTP_OK : GSWMTP_E_HIP;
}

// Kingma and Ba's Adam update with bias-corrected moments, in float32, as one
// inline definition for every kernel that applies it (the plain update, its
// 16-byte form and the one that reads a plan's phase gradient in place), so
// that all of them round alike:
//   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
//   phi -= (lr / (1 - b1^t)) m / (sqrt(v) / sqrt(1 - b2^t) + eps).
#pragma once

#include <hip/hip_runtime.h>

namespace gswmtp {

// Per-step scalars from the step number t: lr / (1 - b1^t) and
// 1 / sqrt(1 - b2^t).
__device__ __forceinline__ void adam_scalars(float t, float lr, float b1, float b2,
                                             float &step_size, float &rbc2) {
  const float bc1 = 1.f - powf(b1, t), bc2 = 1.f - powf(b2, t);
  step_size = lr / bc1;
  rbc2 = 1.f / sqrtf(bc2);
}

// One parameter: moments m, v and the value p updated in place from gradient g.
// The fused multiply-adds are spelled out: left to contraction, the compiler
// fused different products of the same sums in different kernels.
__device__ __forceinline__ void adam_apply(float &p, float &m, float &v, float g, float b1,
                                           float b2, float step_size, float rbc2, float eps) {
  m = fmaf(1.f - b1, g, b1 * m);
  v = fmaf(g, (1.f - b2) * g, b2 * v);
  p -= step_size * m / fmaf(sqrtf(v), rbc2, eps);
}

}  // namespace gswmtp

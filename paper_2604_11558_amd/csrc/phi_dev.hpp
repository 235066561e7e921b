// phi_1 in FP32 for the fused kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace tg {

// phi_1(x) = (e^x - 1) / x.  The arguments here are tau d lambda <= 0 (the
// operators' spectra are real and nonpositive).  For |x| < 1 the Taylor
// series to x^10 / 11! (remainder below 2^-28 relative); below that
// (1 - e^x) / (-x) with the hardware exponential, where 1 - e^x >= 1 - 1/e
// leaves no cancellation (both within about 3 ulp, as expm1f(x) / x).
// Positive arguments take expm1f.
__device__ __forceinline__ float phi1_f32(float x) {
  float t = 1.0f / 39916800.0f;
  t = t * x + 1.0f / 3628800.0f;
  t = t * x + 1.0f / 362880.0f;
  t = t * x + 1.0f / 40320.0f;
  t = t * x + 1.0f / 5040.0f;
  t = t * x + 1.0f / 720.0f;
  t = t * x + 1.0f / 120.0f;
  t = t * x + 1.0f / 24.0f;
  t = t * x + 1.0f / 6.0f;
  t = t * x + 0.5f;
  t = t * x + 1.0f;
  if (x > 1.0f) return expm1f(x) / x;
  const float e = (1.0f - __expf(x)) * __builtin_amdgcn_rcpf(-x);
  return x > -1.0f ? t : e;
}

}  // namespace tg

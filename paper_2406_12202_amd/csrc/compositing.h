// Per-sample arithmetic of the compositing kernels (Eq. 1 and Eq. 5).
#pragma once

#include <hip/hip_runtime.h>

namespace fl {

// Compositing arithmetic of Eq. 1 shared by the compositing kernels, so that
// they round alike: the transmittance e^run (run <= 0, the log-space running
// optical depth) and a sample's opacity 1 - e^-tau (tau >= 0) on the
// hardware base-2 exponential, the opacity below tau = 1/4 by its series to
// tau^7 (truncation below 2e-9 relative), where 1 - e^-tau would cancel; and
// the depth at which the log transmittance l at sample depth t, falling at
// rate sigma, reaches a level (Eq. 5's crossings), by a reciprocal.
__device__ __forceinline__ float transmittance(float run) { return __builtin_amdgcn_exp2f(run * 1.44269504088896341f); }

__device__ __forceinline__ float opacity(float tau) {
  float p = fmaf(tau, 1.0f / 5040.0f, -1.0f / 720.0f);
  p = fmaf(tau, p, 1.0f / 120.0f);
  p = fmaf(tau, p, -1.0f / 24.0f);
  p = fmaf(tau, p, 1.0f / 6.0f);
  p = fmaf(tau, p, -0.5f);
  p = fmaf(tau, p, 1.0f);
  const float series = tau * p;
  const float direct = 1.0f - __builtin_amdgcn_exp2f(-tau * 1.44269504088896341f);
  return tau < 0.25f ? series : direct;
}

__device__ __forceinline__ float crossing_depth(float t, float l, float level, float sigma) {
  return t + (l - level) * __builtin_amdgcn_rcpf(sigma);
}

}  // namespace fl

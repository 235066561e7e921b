// Device side of the steady-state indicators (the integral mean and the L2
// norm of a step's increment): per-point accumulation in an update epilogue
// and the workgroup reduction that stores one partial pair per tile.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace tg {

__device__ __forceinline__ void diag_point(const DiagArgs& d, int rowflat, int col, double nv, double ov,
                                           double& s0, double& s1) {
  const double w = d.w1[col] * d.w23[rowflat];
  const double dl = nv - ov;
  s0 += w * nv;
  s1 += w * dl * dl;
}

// Called by every thread of the workgroup (NW waves) after its last use of
// the LDS area `red` (at least 2 * NW doubles) as tile storage.
template <int NW>
__device__ __forceinline__ void diag_flush(const DiagArgs& d, double s0, double s1, int64_t slot, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s0 += __shfl_xor(s0, off, 64);
    s1 += __shfl_xor(s1, off, 64);
  }
  __syncthreads();
  if (lane == 0) {
    red[2 * wave] = s0;
    red[2 * wave + 1] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t0 = 0.0, t1 = 0.0;
    for (int w = 0; w < NW; ++w) {
      t0 += red[2 * w];
      t1 += red[2 * w + 1];
    }
    d.part[2 * slot] = t0;
    d.part[2 * slot + 1] = t1;
  }
}

}  // namespace tg

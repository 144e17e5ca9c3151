// Work-group sums of the FP64 reductions (energies, overlaps, norms, subspace matrices).
//
// Each wavefront first sums over its 64 lanes with a butterfly of cross-lane moves (no LDS traffic, no
// barrier); the per-wavefront sums then meet in a 16-entry LDS array and every thread adds them in
// wavefront order.  The order of the additions depends only on the launch shape, so a result is the same
// from run to run.  Requirements: blockDim.x a multiple of 64 and at most 1024, and every thread of the
// work-group calls the function (it contains barriers).  Every thread receives the totals.
#pragma once
#include <hip/hip_runtime.h>

namespace tcmi {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ void wg_sum2(double& x, double& y) {
  __shared__ double px[16], py[16];
  x = wave_sum(x);
  y = wave_sum(y);
  const int w = int(threadIdx.x) >> 6, nw = int(blockDim.x) >> 6;
  if ((threadIdx.x & 63) == 0) {
    px[w] = x;
    py[w] = y;
  }
  __syncthreads();
  double sx = 0, sy = 0;
  for (int i = 0; i < nw; ++i) {
    sx += px[i];
    sy += py[i];
  }
  __syncthreads();   // px, py are written again by the next call
  x = sx;
  y = sy;
}

__device__ __forceinline__ double wg_sum(double x) {
  double y = 0;
  wg_sum2(x, y);
  return x;
}

}  // namespace tcmi

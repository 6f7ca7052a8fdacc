// Bounding box of a point set (one workgroup; the searches and the ordering
// that use it read it once per call).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace vecchia_box {

// box[0..D) = per-coordinate minima, box[D..2D) = maxima of locs[n][D]
template <int D>
__global__ void bbox_kernel(int64_t n, const double* __restrict__ locs, double* __restrict__ box) {
  __shared__ double lo[256][D], hi[256][D];
  double l[D], h[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    l[k] = INFINITY;
    h[k] = -INFINITY;
  }
  for (int64_t i = threadIdx.x; i < n; i += 256) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double x = locs[i * D + k];
      l[k] = fmin(l[k], x);
      h[k] = fmax(h[k], x);
    }
  }
#pragma unroll
  for (int k = 0; k < D; ++k) {
    lo[threadIdx.x][k] = l[k];
    hi[threadIdx.x][k] = h[k];
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
#pragma unroll
      for (int k = 0; k < D; ++k) {
        lo[threadIdx.x][k] = fmin(lo[threadIdx.x][k], lo[threadIdx.x + w][k]);
        hi[threadIdx.x][k] = fmax(hi[threadIdx.x][k], hi[threadIdx.x + w][k]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < D) {
    box[threadIdx.x] = lo[0][threadIdx.x];
    box[D + threadIdx.x] = hi[0][threadIdx.x];
  }
}

}  // namespace vecchia_box

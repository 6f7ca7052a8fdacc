// Bounding box of a point set: per-block partial boxes over a grid-stride
// split, then one block over the partials (the searches and the ordering
// read it once per call).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace vecchia_box {

constexpr int kBoxThreads = 256;
constexpr int kBoxMaxBlocks = 1024;

// partial[b][0..D) = minima, partial[b][D..2D) = maxima of the points
// b, b + gridDim.x, ... (in units of kBoxThreads points) of locs[n][D]
template <int D>
__global__ __launch_bounds__(kBoxThreads) void bbox_partial_kernel(int64_t n,
                                                                   const double* __restrict__ locs,
                                                                   double* __restrict__ partial) {
  __shared__ double lo[kBoxThreads][D], hi[kBoxThreads][D];
  double l[D], h[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    l[k] = INFINITY;
    h[k] = -INFINITY;
  }
  for (int64_t i = blockIdx.x * (int64_t)kBoxThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBoxThreads) {
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
  for (int w = kBoxThreads / 2; w > 0; w >>= 1) {
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
    partial[blockIdx.x * 2 * D + threadIdx.x] = lo[0][threadIdx.x];
    partial[blockIdx.x * 2 * D + D + threadIdx.x] = hi[0][threadIdx.x];
  }
}

// box[0..D) = minima, box[D..2D) = maxima over nb partial boxes
template <int D>
__global__ __launch_bounds__(kBoxThreads) void bbox_final_kernel(int nb,
                                                                 const double* __restrict__ partial,
                                                                 double* __restrict__ box) {
  __shared__ double lo[kBoxThreads][D], hi[kBoxThreads][D];
  double l[D], h[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    l[k] = INFINITY;
    h[k] = -INFINITY;
  }
  for (int b = threadIdx.x; b < nb; b += kBoxThreads) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      l[k] = fmin(l[k], partial[b * 2 * D + k]);
      h[k] = fmax(h[k], partial[b * 2 * D + D + k]);
    }
  }
#pragma unroll
  for (int k = 0; k < D; ++k) {
    lo[threadIdx.x][k] = l[k];
    hi[threadIdx.x][k] = h[k];
  }
  __syncthreads();
  for (int w = kBoxThreads / 2; w > 0; w >>= 1) {
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

// Bytes of the partial boxes enqueue_bbox needs.
inline size_t bbox_partial_bytes(int d) { return (size_t)kBoxMaxBlocks * 2 * d * sizeof(double); }

// box[0..2D) of locs[n][D] (n >= 1): per-block partial boxes, then one
// block over them.
template <int D>
inline void enqueue_bbox(int64_t n, const double* locs, double* partial, double* box,
                         hipStream_t st) {
  int64_t nb = (n + kBoxThreads - 1) / kBoxThreads;
  nb = nb < kBoxMaxBlocks ? nb : kBoxMaxBlocks;
  hipLaunchKernelGGL(bbox_partial_kernel<D>, dim3((unsigned)nb), dim3(kBoxThreads), 0, st, n, locs,
                     partial);
  hipLaunchKernelGGL(bbox_final_kernel<D>, dim3(1), dim3(kBoxThreads), 0, st, (int)nb, partial, box);
}

}  // namespace vecchia_box

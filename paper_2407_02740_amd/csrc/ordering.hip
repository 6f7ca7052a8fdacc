// Coarse-to-fine ordering of a point set on the device, an approximation of
// the maxmin ordering the Vecchia approximation is built on (Section 2.1:
// the quality of the conditioning sets depends on the ordering, and maxmin
// orderings, which put every next point as far as possible from those
// already ordered, serve it well).
//
// Each coordinate is quantised to a 2^B grid over the bounding box, with B
// such that a cell holds about one point.  The cell code interleaves the
// grid bits from the most significant down and is then read bit-reversed:
// ordering cells by that value visits a coarse lattice first and fills in
// finer lattices between it.  Several points can share a cell; they are
// ranked within the cell by a tie key, and a point of rank r comes after
// every point of rank r - 1, so each round over the cells is coarse to fine
// again.  The order is the lexicographic one of (rank in cell, reversed
// code, tie key, input index): three stable radix sorts (tie key, reversed
// code, rank) produce it, so it is unique for every input.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "point_box.hpp"
#include "vecchia.h"

namespace vecchia_order {

constexpr int kMaxD = 4;
constexpr int kThreads = 256;

// order-preserving map of a finite double to an unsigned key
__device__ __forceinline__ uint64_t ordered_bits(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  return (b >> 63) ? ~b : (b | (1ull << 63));
}

// rev[i]: grid bits of point i, most significant first, dimension 0 first
// within a level, placed from bit 0 upwards (the bit-reversed cell code);
// tkey[i] = ordered tie bits; idx[i] = i
template <int D>
__global__ void key_kernel(int64_t n, int B, const double* __restrict__ locs,
                           const double* __restrict__ box, const double* __restrict__ tie,
                           uint64_t* __restrict__ rev, uint64_t* __restrict__ tkey,
                           int32_t* __restrict__ idx) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double cells = (double)(1ll << B);
  const int64_t top = (1ll << B) - 1;
  int64_t q[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double lo = box[k];
    const double span = fmax(box[D + k] - lo, 1e-300);
    int64_t c = (int64_t)((locs[i * D + k] - lo) / span * cells);
    q[k] = c < top ? c : top;
  }
  uint64_t r = 0;
  int bit = 0;
  for (int b = B - 1; b >= 0; --b) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      r |= (uint64_t)((q[k] >> b) & 1) << bit;
      ++bit;
    }
  }
  rev[i] = r;
  tkey[i] = ordered_bits(tie[i]);
  idx[i] = (int32_t)i;
}

__global__ void gather_u64_kernel(int64_t n, const uint64_t* __restrict__ src,
                                  const int32_t* __restrict__ idx, uint64_t* __restrict__ dst) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j < n) dst[j] = src[idx[j]];
}

// head[j] = j where a run of equal keys starts, else 0
__global__ void run_head_kernel(int64_t n, const uint64_t* __restrict__ key,
                                uint64_t* __restrict__ head) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j < n) head[j] = (j == 0 || key[j] != key[j - 1]) ? (uint64_t)j : 0;
}

// rank[j] = j - (start of the run j lies in)
__global__ void rank_kernel(int64_t n, const uint64_t* __restrict__ start,
                            uint64_t* __restrict__ rank) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j < n) rank[j] = (uint64_t)j - start[j];
}

template <int D>
__global__ void emit_kernel(int64_t n, const int32_t* __restrict__ idx,
                            const double* __restrict__ locs, int64_t* __restrict__ order,
                            double* __restrict__ locs_out) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t s = idx[j];
  order[j] = s;
  if (locs_out) {
#pragma unroll
    for (int k = 0; k < D; ++k) locs_out[j * D + k] = locs[s * D + k];
  }
}

struct MaxU64 {
  __device__ __host__ uint64_t operator()(uint64_t a, uint64_t b) const { return a > b ? a : b; }
};

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// grid bits per coordinate: about one point per cell, at most 60 code bits
int grid_bits(int64_t n, int d) {
  const double l2 = log2((double)(n > 2 ? n : 2));
  int B = (int)ceil(l2 / d);
  B = B < 1 ? 1 : B;
  return B < 60 / d ? B : 60 / d;
}

struct Work {
  double* box;
  double* box_partial;
  uint64_t *rev, *k0, *k1;
  int32_t *v0, *v1;
  void* sort_tmp;
  size_t sort_bytes;
  void* scan_tmp;
  size_t scan_bytes;
  size_t bytes;
};

// the library's temporary sizes for n items (queried with null storage)
bool tmp_sizes(int64_t n, size_t* sort_bytes, size_t* scan_bytes) {
  rocprim::double_buffer<uint64_t> kb(nullptr, nullptr);
  rocprim::double_buffer<int32_t> vb(nullptr, nullptr);
  size_t a = 0, b = 0;
  if (rocprim::radix_sort_pairs(nullptr, a, kb, vb, (size_t)n, 0u, 64u) != hipSuccess) return false;
  if (rocprim::inclusive_scan(nullptr, b, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                              (size_t)n, MaxU64()) != hipSuccess)
    return false;
  *sort_bytes = a;
  *scan_bytes = b;
  return true;
}

Work carve(void* ws, int64_t n, size_t sort_bytes, size_t scan_bytes) {
  Work w = {};
  char* p = static_cast<char*>(ws);
  size_t o = 0;
  auto take = [&](size_t b) -> char* {
    char* q = p ? p + o : nullptr;
    o += al256(b);
    return q;
  };
  w.box = reinterpret_cast<double*>(take(2 * kMaxD * sizeof(double)));
  w.box_partial = reinterpret_cast<double*>(take(vecchia_box::bbox_partial_bytes(kMaxD)));
  w.rev = reinterpret_cast<uint64_t*>(take(n * sizeof(uint64_t)));
  w.k0 = reinterpret_cast<uint64_t*>(take(n * sizeof(uint64_t)));
  w.k1 = reinterpret_cast<uint64_t*>(take(n * sizeof(uint64_t)));
  w.v0 = reinterpret_cast<int32_t*>(take(n * sizeof(int32_t)));
  w.v1 = reinterpret_cast<int32_t*>(take(n * sizeof(int32_t)));
  w.sort_bytes = sort_bytes;
  w.sort_tmp = take(sort_bytes);
  w.scan_bytes = scan_bytes;
  w.scan_tmp = take(scan_bytes);
  w.bytes = o;
  return w;
}

template <int D>
int run(int64_t n, const double* locs, const double* tie, int64_t* order, double* locs_out,
        Work& w, hipStream_t st) {
  const int B = grid_bits(n, D);
  const unsigned nb = (unsigned)((n + kThreads - 1) / kThreads);
  vecchia_box::enqueue_bbox<D>(n, locs, w.box_partial, w.box, st);
  hipLaunchKernelGGL(key_kernel<D>, dim3(nb), dim3(kThreads), 0, st, n, B, locs, w.box, tie, w.rev,
                     w.k0, w.v0);
  rocprim::double_buffer<uint64_t> keys(w.k0, w.k1);
  rocprim::double_buffer<int32_t> vals(w.v0, w.v1);
  // 1: by tie key
  size_t sb = w.sort_bytes;
  if (rocprim::radix_sort_pairs(w.sort_tmp, sb, keys, vals, (size_t)n, 0u, 64u, st) != hipSuccess)
    return VEC_EHIP;
  // 2: stable by reversed cell code
  hipLaunchKernelGGL(gather_u64_kernel, dim3(nb), dim3(kThreads), 0, st, n, w.rev, vals.current(),
                     keys.current());
  sb = w.sort_bytes;
  if (rocprim::radix_sort_pairs(w.sort_tmp, sb, keys, vals, (size_t)n, 0u, (unsigned)(B * D), st) !=
      hipSuccess)
    return VEC_EHIP;
  // 3: rank within the cell, then stable by rank
  hipLaunchKernelGGL(run_head_kernel, dim3(nb), dim3(kThreads), 0, st, n, keys.current(), w.rev);
  size_t cb = w.scan_bytes;
  if (rocprim::inclusive_scan(w.scan_tmp, cb, (const uint64_t*)w.rev, keys.alternate(), (size_t)n,
                              MaxU64(), st) != hipSuccess)
    return VEC_EHIP;
  hipLaunchKernelGGL(rank_kernel, dim3(nb), dim3(kThreads), 0, st, n, keys.alternate(),
                     keys.current());
  unsigned rbits = 1;
  while (rbits < 63 && (1ll << rbits) < n) ++rbits;
  sb = w.sort_bytes;
  if (rocprim::radix_sort_pairs(w.sort_tmp, sb, keys, vals, (size_t)n, 0u, rbits, st) != hipSuccess)
    return VEC_EHIP;
  hipLaunchKernelGGL(emit_kernel<D>, dim3(nb), dim3(kThreads), 0, st, n, vals.current(), locs,
                     order, locs_out);
  return hipGetLastError() == hipSuccess ? VEC_OK : VEC_EHIP;
}

}  // namespace vecchia_order

using namespace vecchia_order;

extern "C" {

size_t vec_maxmin_order_workspace_bytes(int64_t n, int32_t d) {
  if (n < 1 || n >= (int64_t)INT32_MAX || d < 1 || d > kMaxD) return 0;
  size_t a = 0, b = 0;
  if (!tmp_sizes(n, &a, &b)) return 0;
  return carve(nullptr, n, a, b).bytes;
}

int vec_maxmin_order(int64_t n, int32_t d, const double* locs, const double* tie, int64_t* order,
                     double* locs_out, void* workspace, size_t workspace_bytes, void* stream) {
  if (n < 1 || n >= (int64_t)INT32_MAX || d < 1 || d > kMaxD || !locs || !tie || !order)
    return VEC_EINVAL;
  size_t a = 0, b = 0;
  if (!tmp_sizes(n, &a, &b)) return VEC_EHIP;
  Work w = carve(workspace, n, a, b);
  if (!workspace || workspace_bytes < w.bytes) return VEC_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (d == 1) return run<1>(n, locs, tie, order, locs_out, w, st);
  if (d == 2) return run<2>(n, locs, tie, order, locs_out, w, st);
  if (d == 3) return run<3>(n, locs, tie, order, locs_out, w, st);
  return run<4>(n, locs, tie, order, locs_out, w, st);
}

}  // extern "C"

// Nearest previously ordered neighbours on the device: for every
// observation i of an ordered point set, the min(i, m) observations j < i
// closest to it (Section 2.1: the conditioning sets of the Vecchia
// factorisation), written as NNarray rows [i, nearest, ..., -1 padding].
//
// Observations are taken in doubling blocks [b0, b1) (the first block is
// [0, head)).  For a block, a uniform grid with about per_cell(d) points per
// cell is built over observations [0, b1) (cell ids, counting sort by cell
// with coordinates copied into cell order), and each observation i of the
// block searches the grid in shells of growing Chebyshev radius around its
// own cell, keeping the m best candidates j < i sorted by (distance, index)
// in LDS.  After shell r every point still unvisited lies farther than r
// cell sides, so the search stops once the m-th best distance is below that.
// Candidates within a cell may be visited in any order; the (distance,
// index) order makes the result unique.
//
// With more than four coordinates a grid no longer prunes well; there the
// search is exhaustive (O(n^2) distances): each workgroup of 16 queries (four
// lanes each) walks the earlier points in tiles staged through LDS, keeping
// the same sorted candidate lists, merged per query at the end.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_select.hpp>

#include "point_box.hpp"
#include "vecchia.h"

namespace vecchia_nn {

constexpr int kMaxD = 4;        // grid search
constexpr int kMaxDBrute = 32;  // exhaustive search
constexpr int kQueryThreads = 64;
#ifndef VECCHIA_NN_CELL4
#define VECCHIA_NN_CELL4 3
#endif
// points per grid cell: small cells in one to three dimensions, larger in
// four, where a shell of radius r holds (2r + 1)^4 cells
__host__ __device__ constexpr int per_cell(int d) { return d >= 4 ? VECCHIA_NN_CELL4 : 3; }
constexpr int kMaxM = 64;

struct Grid {
  double lo[kMaxD];
  double side;
  int g[kMaxD];       // cells per dimension
  int64_t stride[kMaxD];
  int64_t ncells;
};

__device__ __forceinline__ int cell_coord(double x, double lo, double side, int g) {
  int c = (int)floor((x - lo) / side);
  return c < 0 ? 0 : (c >= g ? g - 1 : c);
}

__global__ void zero_i32_kernel(int32_t* __restrict__ x, int64_t count) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] = 0;
}

template <int D>
__global__ void cell_kernel(int64_t b1, const double* __restrict__ locs, const Grid g,
                            int32_t* __restrict__ cell, int32_t* __restrict__ count) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= b1) return;
  int64_t c = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) c += (int64_t)cell_coord(locs[j * D + k], g.lo[k], g.side, g.g[k]) * g.stride[k];
  cell[j] = (int32_t)c;
  atomicAdd(&count[c], 1);
}

// cursor[c] = start[c] for the scatter
__global__ void copy_i32_kernel(const int32_t* __restrict__ src, int32_t* __restrict__ dst,
                                int64_t count) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

template <int D>
__global__ void scatter_kernel(int64_t b1, const double* __restrict__ locs,
                               const int32_t* __restrict__ cell, int32_t* __restrict__ cursor,
                               int32_t* __restrict__ sidx, double* __restrict__ sxyz) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= b1) return;
  const int32_t pos = atomicAdd(&cursor[cell[j]], 1);
  sidx[pos] = (int32_t)j;
#pragma unroll
  for (int k = 0; k < D; ++k) sxyz[(int64_t)pos * D + k] = locs[j * D + k];
}

// (d, j) < (e, k) in the order of the result
__device__ __forceinline__ bool before(double d, int32_t j, double e, int32_t k) {
  return d < e || (d == e && j < k);
}

template <int D>
// Queries are taken in grid-cell order (qlist: the block's observations in
// the order of the counting sort), so the lanes of a wave search the same
// neighbourhood of cells.
__global__ __launch_bounds__(kQueryThreads) void query_kernel(
    int64_t nq, const int32_t* __restrict__ qlist, int m, const double* __restrict__ locs,
    const Grid g, const int32_t* __restrict__ start, const int32_t* __restrict__ sidx,
    const double* __restrict__ sxyz, int32_t* __restrict__ NN) {
  // per thread: the m best distances and indices (dynamic LDS, m columns of
  // kQueryThreads entries each)
  extern __shared__ double dyn[];
  double* __restrict__ bdv = dyn;
  int32_t* __restrict__ bjv = reinterpret_cast<int32_t*>(dyn + (size_t)m * kQueryThreads);
  const int t = threadIdx.x;
#define bd(q) bdv[(q) * kQueryThreads + t]
#define bj(q) bjv[(q) * kQueryThreads + t]
  const int64_t qi = blockIdx.x * (int64_t)kQueryThreads + t;
  if (qi >= nq) return;
  const int64_t i = qlist[qi];
  const int me = (int)(i < m ? i : m);
  double xq[D];
  int h[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    xq[k] = locs[i * D + k];
    h[k] = cell_coord(xq[k], g.lo[k], g.side, g.g[k]);
  }
  int cnt = 0;
  double wd = 0.0;
  int32_t wj = 0;
  int gmax = 1;
#pragma unroll
  for (int k = 0; k < D; ++k) gmax = g.g[k] > gmax ? g.g[k] : gmax;
  for (int r = 0; me > 0 && r <= gmax; ++r) {
    // cells at Chebyshev distance exactly r from the home cell
    int o[D];
#pragma unroll
    for (int k = 0; k < D; ++k) o[k] = -r;
    for (;;) {
      bool on_shell = false, inside = true;
      int64_t c = 0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        on_shell = on_shell || o[k] == -r || o[k] == r;
        const int ck = h[k] + o[k];
        inside = inside && ck >= 0 && ck < g.g[k];
        c += (int64_t)ck * g.stride[k];
      }
      if (on_shell && inside) {
        const int32_t pa = start[c], pb = start[c + 1];
        for (int32_t p = pa; p < pb; ++p) {
          const int32_t j = sidx[p];
          if (j >= i) continue;
          double d2 = 0.0;
#pragma unroll
          for (int k = 0; k < D; ++k) {
            const double dz = sxyz[(int64_t)p * D + k] - xq[k];
            d2 = fma(dz, dz, d2);
          }
          if (cnt == me && !before(d2, j, wd, wj)) continue;
          // insert, keeping the list sorted
          int q = (cnt < me) ? cnt : me - 1;
          while (q > 0 && before(d2, j, bd(q - 1), bj(q - 1))) {
            bd(q) = bd(q - 1);
            bj(q) = bj(q - 1);
            --q;
          }
          bd(q) = d2;
          bj(q) = j;
          if (cnt < me) ++cnt;
          if (cnt == me) {  // the current m-th best, kept in registers
            wd = bd(me - 1);
            wj = bj(me - 1);
          }
        }
      }
      // next offset of the cube [-r, r]^D
      int k = 0;
      while (k < D) {
        if (o[k] < r) {
          ++o[k];
          break;
        }
        o[k] = -r;
        ++k;
      }
      if (k == D) break;
    }
    const double reach = r * g.side;
    if (cnt == me && wd < reach * reach) break;
  }
  int32_t* row = NN + i * (int64_t)(m + 1);
  row[0] = (int32_t)i;
  for (int q = 0; q < m; ++q) row[1 + q] = (q < cnt) ? bj(q) : -1;
#undef bd
#undef bj
}

// Exhaustive ordered search for d > 4: 16 queries per workgroup of 64
// lanes, four lanes per query splitting the candidates j < i (lane part p
// takes j = p (mod 4) of every tile), candidates in tiles of 64 points
// staged through LDS (tile[64][d]); each lane keeps a sorted list as in
// query_kernel, and the first lane of a query merges the four lists.
constexpr int kBruteQueries = 16;
constexpr int kBruteSplit = kQueryThreads / kBruteQueries;

__global__ __launch_bounds__(kQueryThreads) void brute_kernel(int64_t n, int d, int m,
                                                              const double* __restrict__ locs,
                                                              int32_t* __restrict__ NN) {
  extern __shared__ double dyn[];
  double* __restrict__ tile = dyn;                                 // [kQueryThreads][d]
  double* __restrict__ xq = dyn + (size_t)kQueryThreads * d;        // [kBruteQueries][d]
  double* __restrict__ bdv = xq + (size_t)kBruteQueries * d;         // [m][kQueryThreads]
  int32_t* __restrict__ bjv = reinterpret_cast<int32_t*>(bdv + (size_t)(m > 0 ? m : 1) * kQueryThreads);
  int32_t* __restrict__ cnts = bjv + (size_t)(m > 0 ? m : 1) * kQueryThreads;  // [kQueryThreads]
  const int t = threadIdx.x;
  const int qloc = t / kBruteSplit, part = t % kBruteSplit;
#define bd(q) bdv[(q) * kQueryThreads + t]
#define bj(q) bjv[(q) * kQueryThreads + t]
  const int64_t i0 = blockIdx.x * (int64_t)kBruteQueries;
  const int64_t i = i0 + qloc;
  const bool live = i < n;
  const int me = live ? (int)(i < m ? i : m) : 0;
  for (int e = t; e < kBruteQueries * d; e += kQueryThreads) {
    const int64_t iq = i0 + e / d;
    xq[e] = (iq < n) ? locs[iq * d + e % d] : 0.0;
  }
  int cnt = 0;
  double wd = 0.0;
  int32_t wj = 0;
  const int64_t jend = (i0 + kBruteQueries < n) ? i0 + kBruteQueries : n;  // candidates < jend
  for (int64_t j0 = 0; j0 < jend; j0 += kQueryThreads) {
    const int64_t tn = (jend - j0 < kQueryThreads) ? jend - j0 : kQueryThreads;
    __syncthreads();
    for (int64_t e = t; e < tn * d; e += kQueryThreads) tile[e] = locs[j0 * d + e];
    __syncthreads();
    if (me > 0) {
      for (int jj = part; jj < (int)tn; jj += kBruteSplit) {
        const int64_t j = j0 + jj;
        if (j >= i) break;
        double d2 = 0.0;
        for (int k = 0; k < d; ++k) {
          const double dz = tile[jj * d + k] - xq[qloc * d + k];
          d2 = fma(dz, dz, d2);
        }
        if (cnt == me && !before(d2, (int32_t)j, wd, wj)) continue;
        int q = (cnt < me) ? cnt : me - 1;
        while (q > 0 && before(d2, (int32_t)j, bd(q - 1), bj(q - 1))) {
          bd(q) = bd(q - 1);
          bj(q) = bj(q - 1);
          --q;
        }
        bd(q) = d2;
        bj(q) = (int32_t)j;
        if (cnt < me) ++cnt;
        if (cnt == me) {
          wd = bd(me - 1);
          wj = bj(me - 1);
        }
      }
    }
  }
  cnts[t] = cnt;
  __syncthreads();
  if (live && part == 0) {
    // merge the query's four sorted lists (disjoint candidate sets)
    int pos[kBruteSplit], len[kBruteSplit];
    for (int p = 0; p < kBruteSplit; ++p) {
      pos[p] = 0;
      len[p] = cnts[t + p];
    }
    int32_t* row = NN + i * (int64_t)(m + 1);
    row[0] = (int32_t)i;
    for (int q = 0; q < m; ++q) {
      int best = -1;
      double bdist = 0.0;
      int32_t bidx = 0;
      for (int p = 0; p < kBruteSplit; ++p) {
        if (pos[p] < len[p]) {
          const double dp = bdv[pos[p] * kQueryThreads + t + p];
          const int32_t jp = bjv[pos[p] * kQueryThreads + t + p];
          if (best < 0 || before(dp, jp, bdist, bidx)) {
            best = p;
            bdist = dp;
            bidx = jp;
          }
        }
      }
      if (q < me && best >= 0) {
        row[1 + q] = bidx;
        ++pos[best];
      } else {
        row[1 + q] = -1;
      }
    }
  }
#undef bd
#undef bj
}

}  // namespace vecchia_nn

using namespace vecchia_nn;

namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t head_of(int64_t n, int m) {
  const int64_t h = 4 * (int64_t)(m + 1) > 64 ? 4 * (int64_t)(m + 1) : 64;
  return h < n ? h : n;
}

// the largest cell count any block's grid can have
int64_t max_cells(int64_t n, int d) { return n / per_cell(d) + 8 * 8 * 8 * 8 + 1; }

struct Work {
  double* box;
  double* box_partial;
  void* scan_tmp;
  size_t scan_bytes;
  void* sel_tmp;
  size_t sel_bytes;
  int32_t* qlist;
  int64_t* qcount;
  int32_t *cell, *count, *start, *cursor, *sidx;
  double* sxyz;
  size_t bytes;
};

// the library's temporary bytes of an exclusive scan of `count` int32 values
size_t scan_bytes_for(int64_t count) {
  size_t b = 0;
  if (rocprim::exclusive_scan(nullptr, b, (const int32_t*)nullptr, (int32_t*)nullptr, 0,
                              (size_t)count, rocprim::plus<int32_t>()) != hipSuccess)
    return 0;
  return b;
}

struct AtLeast {
  int32_t lo;
  __device__ __host__ bool operator()(int32_t j) const { return j >= lo; }
};

// the library's temporary bytes of selecting from `count` int32 values
size_t select_bytes_for(int64_t count) {
  size_t b = 0;
  if (rocprim::select(nullptr, b, (const int32_t*)nullptr, (int32_t*)nullptr, (int64_t*)nullptr,
                      (size_t)count, AtLeast{0}) != hipSuccess)
    return 0;
  return b;
}

Work carve(void* ws, int64_t n, int d) {
  Work w = {};
  char* p = static_cast<char*>(ws);
  size_t o = 0;
  auto take = [&](size_t b) -> char* {
    char* q = p ? p + o : nullptr;
    o += al256(b);
    return q;
  };
  const int64_t nc = max_cells(n, d);
  w.box = reinterpret_cast<double*>(take(2 * kMaxD * sizeof(double)));
  w.box_partial = reinterpret_cast<double*>(take(vecchia_box::bbox_partial_bytes(kMaxD)));
  w.scan_bytes = scan_bytes_for(nc + 1);
  w.scan_tmp = take(w.scan_bytes);
  w.sel_bytes = select_bytes_for(n);
  w.sel_tmp = take(w.sel_bytes);
  w.qlist = reinterpret_cast<int32_t*>(take(n * sizeof(int32_t)));
  w.qcount = reinterpret_cast<int64_t*>(take(sizeof(int64_t)));
  w.cell = reinterpret_cast<int32_t*>(take(n * sizeof(int32_t)));
  w.count = reinterpret_cast<int32_t*>(take((nc + 1) * sizeof(int32_t)));
  w.start = reinterpret_cast<int32_t*>(take((nc + 1) * sizeof(int32_t)));
  w.cursor = reinterpret_cast<int32_t*>(take((nc + 1) * sizeof(int32_t)));
  w.sidx = reinterpret_cast<int32_t*>(take(n * sizeof(int32_t)));
  w.sxyz = reinterpret_cast<double*>(take((size_t)n * d * sizeof(double)));
  w.bytes = o;
  return w;
}

// grid over points [0, b1) inside the box: equal cell sides, about per_cell(d)
// points per cell (dimensions of negligible extent get one cell)
Grid make_grid(const double* lo, const double* hi, int d, int64_t b1) {
  Grid g = {};
  double ext[kMaxD], emax = 0.0;
  for (int k = 0; k < d; ++k) {
    ext[k] = hi[k] - lo[k];
    emax = ext[k] > emax ? ext[k] : emax;
  }
  double vol = 1.0;
  int dd = 0;
  for (int k = 0; k < d; ++k) {
    if (ext[k] > 1e-12 * emax) {
      vol *= ext[k];
      ++dd;
    }
  }
  const double target = (double)(b1 / per_cell(d) > 1 ? b1 / per_cell(d) : 1);
  double side = (dd > 0 && vol > 0.0) ? pow(vol / target, 1.0 / dd) : 1.0;
  if (!(side > 0.0)) side = 1.0;
  int64_t nc = 1;
  for (int k = 0; k < d; ++k) {
    int gk = (ext[k] > 1e-12 * emax) ? (int)ceil(ext[k] / side) : 1;
    gk = gk < 1 ? 1 : gk;
    g.g[k] = gk;
    g.lo[k] = lo[k];
    nc *= gk;
  }
  // the rounding up can overshoot the target; widen until within bounds
  while (nc > max_cells(b1, d) - 1) {
    side *= 1.1;
    nc = 1;
    for (int k = 0; k < d; ++k) {
      int gk = (ext[k] > 1e-12 * emax) ? (int)ceil(ext[k] / side) : 1;
      g.g[k] = gk < 1 ? 1 : gk;
      nc *= g.g[k];
    }
  }
  g.side = side;
  int64_t st = 1;
  for (int k = 0; k < d; ++k) {
    g.stride[k] = st;
    st *= g.g[k];
  }
  g.ncells = st;
  return g;
}

template <int D>
int run(int64_t n, int m, const double* locs, int32_t* NN, const Work& w, hipStream_t st) {
  vecchia_box::enqueue_bbox<D>(n, locs, w.box_partial, w.box, st);
  double box[2 * kMaxD];
  if (hipMemcpyAsync(box, w.box, 2 * D * sizeof(double), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return VEC_EHIP;
  for (int k = 0; k < D; ++k)
    if (!isfinite(box[k]) || !isfinite(box[D + k])) return VEC_EINVAL;
  int64_t b0 = 0, b1 = head_of(n, m);
  while (b0 < n) {
    const Grid g = make_grid(box, box + D, D, b1);
    const unsigned nb = (unsigned)((b1 + 255) / 256);
    hipLaunchKernelGGL(zero_i32_kernel, dim3(256), dim3(256), 0, st, w.count, g.ncells + 1);
    hipLaunchKernelGGL(cell_kernel<D>, dim3(nb), dim3(256), 0, st, b1, locs, g, w.cell, w.count);
    // start[c] = sum of count[0..c), start[ncells] = the total; cursor = start
    size_t sb = w.scan_bytes;
    if (rocprim::exclusive_scan(w.scan_tmp, sb, (const int32_t*)w.count, w.start, 0,
                                (size_t)(g.ncells + 1), rocprim::plus<int32_t>(), st) != hipSuccess)
      return VEC_EHIP;
    hipLaunchKernelGGL(copy_i32_kernel, dim3(256), dim3(256), 0, st, w.start, w.cursor,
                       g.ncells + 1);
    hipLaunchKernelGGL(scatter_kernel<D>, dim3(nb), dim3(256), 0, st, b1, locs, w.cell, w.cursor,
                       w.sidx, w.sxyz);
    const unsigned nq = (unsigned)((b1 - b0 + kQueryThreads - 1) / kQueryThreads);
    const size_t lds = (size_t)(m > 0 ? m : 1) * kQueryThreads * (sizeof(double) + sizeof(int32_t));
    // the block's observations (indices >= b0) in cell order
    size_t sb2 = w.sel_bytes;
    if (rocprim::select(w.sel_tmp, sb2, (const int32_t*)w.sidx, w.qlist, w.qcount, (size_t)b1,
                        AtLeast{(int32_t)b0}, st) != hipSuccess)
      return VEC_EHIP;
    hipLaunchKernelGGL(query_kernel<D>, dim3(nq), dim3(kQueryThreads), lds, st, b1 - b0, w.qlist,
                       m, locs, g, w.start, w.sidx, w.sxyz, NN);
    if (hipGetLastError() != hipSuccess) return VEC_EHIP;
    b0 = b1;
    b1 = 2 * b1 < n ? 2 * b1 : n;
  }
  return VEC_OK;
}

}  // namespace

extern "C" {

size_t vec_ordered_nn_workspace_bytes(int64_t n, int32_t d, int32_t m) {
  if (n < 1 || n >= (int64_t)INT32_MAX || d < 1 || d > kMaxDBrute || m < 0 || m > kMaxM) return 0;
  if (d > kMaxD) return 256;  // the exhaustive search needs none; a token size
  return carve(nullptr, n, d).bytes;
}

int vec_ordered_nn(int64_t n, int32_t d, int32_t m, const double* locs, int32_t* NNarray,
                   void* workspace, size_t workspace_bytes, void* stream) {
  if (n < 1 || n >= (int64_t)INT32_MAX || d < 1 || d > kMaxDBrute || m < 0 || m > kMaxM ||
      !locs || !NNarray)
    return VEC_EINVAL;
  const size_t need = vec_ordered_nn_workspace_bytes(n, d, m);
  if (!workspace || workspace_bytes < need) return VEC_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (d > kMaxD) {
    const unsigned nb = (unsigned)((n + kBruteQueries - 1) / kBruteQueries);
    const size_t lds = ((size_t)(kQueryThreads + kBruteQueries) * d +
                        (size_t)(m > 0 ? m : 1) * kQueryThreads) *
                           sizeof(double) +
                       ((size_t)(m > 0 ? m : 1) + 1) * kQueryThreads * sizeof(int32_t);
    if (lds > 65536) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(brute_kernel),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds);
      if (e != hipSuccess) return VEC_EHIP;
    }
    hipLaunchKernelGGL(brute_kernel, dim3(nb), dim3(kQueryThreads), lds, st, n, (int)d, (int)m,
                       locs, NNarray);
    return hipGetLastError() == hipSuccess ? VEC_OK : VEC_EHIP;
  }
  const Work w = carve(workspace, n, d);
  if (d == 1) return run<1>(n, m, locs, NNarray, w, st);
  if (d == 2) return run<2>(n, m, locs, NNarray, w, st);
  if (d == 3) return run<3>(n, m, locs, NNarray, w, st);
  return run<4>(n, m, locs, NNarray, w, st);
}

}  // extern "C"

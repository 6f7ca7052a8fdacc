// C ABI of the Vecchia library (declarations and contract in vecchia.h) and
// the small single-workgroup kernels around the fused per-neighbourhood
// kernel: the fixed-order reduction of workgroup partials, the combine step
// ("separate function", Section 3), the Fisher-scoring update (Eq. 4) and
// the status word.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "vecchia.h"
#include "vecchia_wave.hpp"
#include "vecchia_kernels.hpp"

namespace vecchia {

#ifdef VECCHIA_SECTION_TIMING
__device__ unsigned long long section_cycles[kSections];
#endif

// Instantiations live in vecchia_inst_k*.hip (compiled in parallel).
#define VEC_DECLARE(K, PC, NG, MODE, B)                 \
  extern template VECCHIA_LAUNCH_SIG(K, PC, NG, MODE, B); \
  extern template VECCHIA_RESIDENT_SIG(K, PC, NG, MODE, B)
#define VEC_DECLARE_K(K)                   \
  VECCHIA_FOR_MODES(VEC_DECLARE, K, 1);    \
  VECCHIA_FOR_MODES(VEC_DECLARE, K, 2);    \
  VECCHIA_FOR_MODES(VEC_DECLARE, K, 3)
VEC_DECLARE_K(11);
VEC_DECLARE_K(21);
VEC_DECLARE_K(31);
VEC_DECLARE_K(41);
#define VEC_DECLARE_SINGLE(K, PC, NG, MODE, B) extern template VECCHIA_LAUNCH_SIG(K, PC, NG, MODE, B)
VECCHIA_FOR_SINGLE(VEC_DECLARE_SINGLE, 35, 1);
VECCHIA_FOR_SINGLE(VEC_DECLARE_SINGLE, 35, 2);
VECCHIA_FOR_SINGLE(VEC_DECLARE_SINGLE, 35, 3);
VECCHIA_FOR_SINGLE(VEC_DECLARE_SINGLE, 61, 1);
VECCHIA_FOR_SINGLE(VEC_DECLARE_SINGLE, 61, 2);
VECCHIA_FOR_SINGLE(VEC_DECLARE_SINGLE, 61, 3);

// kLaunch[K index][p - 1][space-time][mode]: single problem
#define VEC_NG(K, PC, NG)                                                                   \
  {launch_sums<K, PC, NG, kModeSums, false>, launch_sums<K, PC, NG, kModeAdjoint, false>, \
   launch_sums<K, PC, NG, kModeLoglik, false>, launch_sums<K, PC, NG, kModeWeights, false>}
#define VEC_PC(K, PC) {VEC_NG(K, PC, 1), VEC_NG(K, PC, 2)}
#define VEC_ROW(K) {VEC_PC(K, 1), VEC_PC(K, 2), VEC_PC(K, 3)}
constexpr int kNumModes = 4;
static const launch_fn kLaunch[kNumK][3][2][kNumModes] = {
    VEC_ROW(11), VEC_ROW(21), VEC_ROW(31), VEC_ROW(35), VEC_ROW(41), VEC_ROW(61)};
// kLaunchBatch / kResidentBatch[K index][p - 1][space-time]: batched sums
#define VEC_BPC(K, PC, F) {F<K, PC, 1, kModeSums, true>, F<K, PC, 2, kModeSums, true>}
#define VEC_BROW(K, F) {VEC_BPC(K, 1, F), VEC_BPC(K, 2, F), VEC_BPC(K, 3, F)}
static const launch_fn kLaunchBatch[kNumBatchK][3][2] = {
    VEC_BROW(11, launch_sums), VEC_BROW(21, launch_sums), VEC_BROW(31, launch_sums),
    VEC_BROW(41, launch_sums)};
static const resident_fn kResidentBatch[kNumBatchK][3][2] = {
    VEC_BROW(11, resident_sums), VEC_BROW(21, resident_sums), VEC_BROW(31, resident_sums),
    VEC_BROW(41, resident_sums)};

#ifndef VECCHIA_BLOCKS_PER_CU
#define VECCHIA_BLOCKS_PER_CU 8
#endif
// Grid of the single-problem launches: workgroups per CU (twice the resident
// count at K <= 31, so a second round of workgroups fills in behind the first).
constexpr int kBlocksPerCU = VECCHIA_BLOCKS_PER_CU;
constexpr int kMaxP = 3;
constexpr int kMaxParms = 4;                            // fused-kernel families
constexpr int kMaxParmsAniso = vecchia_wave::kMaxD + 2;  // one range per coordinate

struct Dims {
  int p, P, nraw, nout, kidx, nu;
  bool wave;  // the wave-per-neighbourhood kernel (one range per coordinate, or m + 1 > 41)
};

static bool dims_of(const vec_problem* pb, Dims* dm) {
  if (!pb) return false;
  if (pb->n < 1 || pb->n >= (int64_t)INT32_MAX) return false;
  if (pb->m < 0 || pb->d < 1 || pb->p < 1 || pb->p > kMaxP) return false;
  if (pb->reserved != 0) return false;
  dm->wave = false;
  if (pb->family == VEC_FAMILY_ISO) {
    if (pb->d > 4) return false;
    dm->P = 3;
  } else if (pb->family == VEC_FAMILY_SPACETIME) {
    if (pb->d > 4 || pb->nspace < 1 || pb->nspace >= pb->d) return false;
    dm->P = 4;
    // the fused kernel scales the last coordinate alone by rho_t; any other
    // split of the coordinates runs on the wave kernel
    if (pb->nspace != pb->d - 1) {
      if (pb->m + 1 > vecchia_wave::kMaxK) return false;
      dm->wave = true;
    }
  } else if (pb->family == VEC_FAMILY_ANISO) {
    if (pb->d > vecchia_wave::kMaxD || pb->m + 1 > vecchia_wave::kMaxK) return false;
    dm->P = pb->d + 2;
    dm->wave = true;
  } else {
    return false;
  }
  if (pb->smoothness == 0.5)
    dm->nu = 0;
  else if (pb->smoothness == 1.5)
    dm->nu = 1;
  else if (pb->smoothness == 2.5)
    dm->nu = 2;
  else
    return false;
  dm->kidx = -1;
  for (int k = 0; k < kNumK; ++k) {
    if (pb->m + 1 <= kKs[k]) {
      dm->kidx = k;
      break;
    }
  }
  if (dm->kidx < 0) {
    // neighbourhoods beyond the fused kernel's sizes: the wave kernel
    if (pb->m + 1 > vecchia_wave::kMaxK) return false;
    dm->wave = true;
  }
  dm->p = pb->p;
  dm->nraw = nraw_of(dm->p, dm->P);
  dm->nout = 1 + dm->P + dm->P * dm->P + dm->p + dm->p * dm->p;
  return true;
}

static int grid_for(int64_t total) {
  if (total <= 0) return 0;
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      ncu = v;
  }
  const int64_t want = (total + kGroupsPerBlock - 1) / kGroupsPerBlock;
  const int64_t cap = (int64_t)ncu * kBlocksPerCU;
  return (int)(want < cap ? want : cap);
}

// ----------------------------------------------------------------------------
// small kernels
// ----------------------------------------------------------------------------

// raw[e] = sum over blocks of partials[b][e], one workgroup per entry, fixed
// strided assignment and fixed tree: deterministic.
__global__ __launch_bounds__(256) void reduce_kernel(const double* __restrict__ partials, int nblocks,
                                                     int nraw, double* __restrict__ raw) {
  __shared__ double red[256];
  const int e = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 256) s += partials[(size_t)b * nraw + e];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) raw[e] = red[0];
}

// Kriging prediction from the weights of the prediction rows: for row j
// (observation n_obs + j of the augmented problem) with weights b over its
// neighbours s and w[m] = log(v / sigma2),
//   mean_j = x_j beta + sum_l b_l (y_s_l - x_s_l beta),  var_j = sigma2 e^w[m].
__global__ void predict_kernel(int64_t n_obs, int64_t n_pred, int m, int p,
                               const int32_t* __restrict__ NN, const double* __restrict__ y,
                               const double* __restrict__ X, const double* __restrict__ beta,
                               const double* __restrict__ covparms,
                               const double* __restrict__ w, double* __restrict__ mean,
                               double* __restrict__ var) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n_pred) return;
  const int64_t i = n_obs + j;
  const int32_t* row = NN + j * (int64_t)(m + 1);
  const double* wj = w + j * (int64_t)(m + 1);
  double mu = 0.0;
  for (int t = 0; t < p; ++t) mu += X[i * p + t] * beta[t];
  for (int l = 0; l < m; ++l) {
    const int64_t s = row[1 + l];
    if (s < 0 || s >= n_obs) continue;  // malformed row: flagged by the weights pass
    double r = y[s];
    for (int t = 0; t < p; ++t) r -= X[s * p + t] * beta[t];
    mu += wj[l] * r;
  }
  mean[j] = mu;
  var[j] = covparms[0] * exp(wj[m]);
}

// sum[e] = a[e] + b[e] (b may be null)
__global__ void add_raw_kernel(const double* __restrict__ a, const double* __restrict__ b, int count,
                               double* __restrict__ sum) {
  for (int e = threadIdx.x; e < count; e += blockDim.x) sum[e] = b ? a[e] + b[e] : a[e];
}

__global__ void fill_kernel(double* __restrict__ x, int count, double v) {
  for (int e = threadIdx.x; e < count; e += blockDim.x) x[e] = v;
}

__global__ void status_clear_kernel(int32_t* status) {
  if (threadIdx.x == 0) {
    status[0] = 0;
    status[1] = INT32_MAX;
  }
}

// Cholesky of a small SPD matrix in place (row-major, lower), false if not PD.
__device__ bool small_chol(double* a, int k) {
  for (int r = 0; r < k; ++r) {
    for (int c = 0; c <= r; ++c) {
      double s = a[r * k + c];
      for (int t = 0; t < c; ++t) s -= a[r * k + t] * a[c * k + t];
      if (r == c) {
        if (!(s > 0.0)) return false;
        a[r * k + r] = sqrt(s);
      } else {
        a[r * k + c] = s / a[c * k + c];
      }
    }
  }
  return true;
}

__device__ void small_chol_solve(const double* L, int k, double* x) {
  for (int r = 0; r < k; ++r) {
    double s = x[r];
    for (int t = 0; t < r; ++t) s -= L[r * k + t] * x[t];
    x[r] = s / L[r * k + r];
  }
  for (int r = k - 1; r >= 0; --r) {
    double s = x[r];
    for (int t = r + 1; t < k; ++t) s -= L[t * k + r] * x[t];
    x[r] = s / L[r * k + r];
  }
}

// The "separate function" of Section 3 (profile over beta by generalised
// least squares).
__device__ void combine_one(int64_t n, int p, int P, const double* __restrict__ raw,
                            double* __restrict__ out, int32_t* __restrict__ status) {
  const double logdet = raw[0], ySy = raw[1];
  const double* XSX = raw + 2;
  const double* ySX = XSX + p * p;
  const double* dlogdet = ySX + p;
  const double* dySy = dlogdet + P;
  const double* dXSX = dySy + P;
  const double* dySX = dXSX + P * p * p;
  const double* ainfo = dySX + P * p;
  double L[kMaxP * kMaxP], beta[kMaxP];
  for (int e = 0; e < p * p; ++e) L[e] = XSX[e];
  for (int t = 0; t < p; ++t) beta[t] = ySX[t];
  bool ok = small_chol(L, p);
  if (ok) small_chol_solve(L, p, beta);
  double quad = ySy;
  for (int t = 0; t < p; ++t) quad -= ySX[t] * beta[t];
  double* o = out;
  *o++ = -0.5 * ((double)n * log(2.0 * M_PI) + logdet + quad);
  for (int j = 0; j < P; ++j) {
    double g = dlogdet[j] + dySy[j];
    for (int t = 0; t < p; ++t) g -= 2.0 * beta[t] * dySX[j * p + t];
    for (int s = 0; s < p; ++s)
      for (int t = 0; t < p; ++t) g += beta[s] * dXSX[(j * p + s) * p + t] * beta[t];
    *o++ = -0.5 * g;
  }
  for (int e = 0; e < P * P; ++e) *o++ = ainfo[e];
  for (int t = 0; t < p; ++t) *o++ = beta[t];
  for (int e = 0; e < p * p; ++e) *o++ = XSX[e];
  bool finite = ok;
  for (int e = 0; e < 1 + P; ++e) finite = finite && __builtin_isfinite(out[e]);
  if (!finite) {
    atomicOr(&status[0], VEC_FLAG_NONFINITE);
  }
}

__global__ void combine_kernel(int64_t n, int p, int P, const double* __restrict__ raw,
                               double* __restrict__ out, int32_t* __restrict__ status) {
  if (threadIdx.x == 0) combine_one(n, p, P, raw, out, status);
}

// Eq. (4) on the log scale with a step-length cap (P <= MAXP).
template <int MAXP>
__device__ void fisher_one(int P, const double* __restrict__ out, double* __restrict__ covparms,
                           int32_t* __restrict__ status, double max_step) {
  if (status[0] != 0) return;
  const double* grad = out + 1;
  const double* info = grad + P;
  double th[MAXP], g[MAXP], I[MAXP * MAXP];
  for (int j = 0; j < P; ++j) {
    th[j] = covparms[j];
    g[j] = th[j] * grad[j];
  }
  for (int j = 0; j < P; ++j)
    for (int k = 0; k < P; ++k) I[j * P + k] = th[j] * info[j * P + k] * th[k];
  if (!small_chol(I, P)) {
    atomicOr(&status[0], VEC_FLAG_NONFINITE);
    return;
  }
  small_chol_solve(I, P, g);
  double norm2 = 0.0;
  for (int j = 0; j < P; ++j) norm2 += g[j] * g[j];
  const double norm = sqrt(norm2);
  const double scale = (norm > max_step) ? max_step / norm : 1.0;
  for (int j = 0; j < P; ++j) covparms[j] = th[j] * exp(g[j] * scale);
}

template <int MAXP>
__global__ void fisher_kernel(int P, const double* __restrict__ out,
                              double* __restrict__ covparms, int32_t* __restrict__ status,
                              double max_step) {
  if (threadIdx.x == 0) fisher_one<MAXP>(P, out, covparms, status, max_step);
}

// The same update for many parameters, spread over one 64-lane workgroup:
// the scaled information in LDS, a right-looking Cholesky with the rows of
// each column step split over the lanes, and column-sweep substitutions.
template <int MAXP>
__global__ __launch_bounds__(64) void fisher_wide_kernel(int P, const double* __restrict__ out,
                                                         double* __restrict__ covparms,
                                                         int32_t* __restrict__ status,
                                                         double max_step) {
  __shared__ double I[MAXP][MAXP + 1];
  __shared__ double g[MAXP], th[MAXP];
  __shared__ int fail;
  const int t = threadIdx.x;
  if (status[0] != 0) return;  // the same word for every lane
  const double* grad = out + 1;
  const double* info = grad + P;
  if (t == 0) fail = 0;
  for (int j = t; j < P; j += 64) {
    th[j] = covparms[j];
    g[j] = th[j] * grad[j];
  }
  __syncthreads();
  for (int e = t; e < P * P; e += 64) {
    const int j = e / P, k = e % P;
    I[j][k] = th[j] * info[e] * th[k];
  }
  __syncthreads();
  for (int c = 0; c < P; ++c) {
    if (t == 0) {
      const double piv = I[c][c];
      if (!(piv > 0.0)) fail = 1;
      I[c][c] = sqrt(piv);
    }
    __syncthreads();
    if (fail) break;  // the same value for every lane
    for (int r = c + 1 + t; r < P; r += 64) I[r][c] /= I[c][c];
    __syncthreads();
    const int w = P - c - 1;
    for (int e = t; e < w * w; e += 64) {
      const int r = c + 1 + e / w, s2 = c + 1 + e % w;
      if (s2 <= r) I[r][s2] -= I[r][c] * I[s2][c];
    }
    __syncthreads();
  }
  if (fail) {
    if (t == 0) atomicOr(&status[0], VEC_FLAG_NONFINITE);
    return;
  }
  for (int c = 0; c < P; ++c) {  // L y = g
    if (t == 0) g[c] /= I[c][c];
    __syncthreads();
    for (int r = c + 1 + t; r < P; r += 64) g[r] -= I[r][c] * g[c];
    __syncthreads();
  }
  for (int c = P - 1; c >= 0; --c) {  // L^T x = y
    if (t == 0) g[c] /= I[c][c];
    __syncthreads();
    for (int r = t; r < c; r += 64) g[r] -= I[c][r] * g[c];
    __syncthreads();
  }
  double norm2 = 0.0;
  for (int j = 0; j < P; ++j) norm2 += g[j] * g[j];
  const double norm = sqrt(norm2);
  const double scale = (norm > max_step) ? max_step / norm : 1.0;
  for (int j = t; j < P; j += 64) covparms[j] = th[j] * exp(g[j] * scale);
}

// The combine step spread over one workgroup (many parameters): the GLS
// solve and the log-likelihood on lane 0, gradient entries and copies of the
// information over the lanes.
__global__ __launch_bounds__(64) void combine_wide_kernel(int64_t n, int p, int P,
                                                          const double* __restrict__ raw,
                                                          double* __restrict__ out,
                                                          int32_t* __restrict__ status) {
  __shared__ double beta[kMaxP];
  __shared__ int ok;
  const int t = threadIdx.x;
  const double logdet = raw[0], ySy = raw[1];
  const double* XSX = raw + 2;
  const double* ySX = XSX + p * p;
  const double* dlogdet = ySX + p;
  const double* dySy = dlogdet + P;
  const double* dXSX = dySy + P;
  const double* dySX = dXSX + P * p * p;
  const double* ainfo = dySX + P * p;
  if (t == 0) {
    double L[kMaxP * kMaxP], b[kMaxP];
    for (int e = 0; e < p * p; ++e) L[e] = XSX[e];
    for (int j = 0; j < p; ++j) b[j] = ySX[j];
    ok = small_chol(L, p) ? 1 : 0;
    if (ok) small_chol_solve(L, p, b);
    double quad = ySy;
    for (int j = 0; j < p; ++j) {
      quad -= ySX[j] * b[j];
      beta[j] = b[j];
    }
    out[0] = -0.5 * ((double)n * log(2.0 * M_PI) + logdet + quad);
  }
  __syncthreads();
  bool finite = true;
  for (int j = t; j < P; j += 64) {
    double gj = dlogdet[j] + dySy[j];
    for (int a = 0; a < p; ++a) gj -= 2.0 * beta[a] * dySX[j * p + a];
    for (int a = 0; a < p; ++a)
      for (int b = 0; b < p; ++b) gj += beta[a] * dXSX[(j * p + a) * p + b] * beta[b];
    out[1 + j] = -0.5 * gj;
    finite = finite && __builtin_isfinite(gj);
  }
  for (int e = t; e < P * P; e += 64) out[1 + P + e] = ainfo[e];
  for (int j = t; j < p; j += 64) out[1 + P + P * P + j] = beta[j];
  for (int e = t; e < p * p; e += 64) out[1 + P + P * P + p + e] = XSX[e];
  if (t == 0) finite = finite && ok && __builtin_isfinite(out[0]);
  if (!finite) atomicOr(&status[0], VEC_FLAG_NONFINITE);
}

static void enqueue_fisher(const Dims& dm, const double* out, double* covparms, int32_t* status,
                           double max_step, hipStream_t st) {
  if (dm.P <= kMaxParms)
    hipLaunchKernelGGL(fisher_kernel<kMaxParms>, dim3(1), dim3(64), 0, st, dm.P, out, covparms,
                       status, max_step);
  else
    hipLaunchKernelGGL(fisher_wide_kernel<kMaxParmsAniso>, dim3(1), dim3(64), 0, st, dm.P, out,
                       covparms, status, max_step);
}

static void enqueue_combine(const vec_problem* pb, const Dims& dm, const double* raw, double* out,
                            int32_t* status, hipStream_t st) {
  if (dm.P <= kMaxParms)
    hipLaunchKernelGGL(combine_kernel, dim3(1), dim3(64), 0, st, pb->n, dm.p, dm.P, raw, out,
                       status);
  else
    hipLaunchKernelGGL(combine_wide_kernel, dim3(1), dim3(64), 0, st, pb->n, dm.p, dm.P, raw, out,
                       status);
}

// ----------------------------------------------------------------------------
// batches of datasets
// ----------------------------------------------------------------------------

// raw[b][e] = sum of dataset b's partial rows (its tiles, in tile order),
// one workgroup per (entry, dataset), fixed tree: deterministic.
__global__ __launch_bounds__(256) void batch_reduce_kernel(const int64_t* __restrict__ sets,
                                                           const double* __restrict__ partials,
                                                           int nraw, double* __restrict__ raw) {
  __shared__ double red[256];
  const int e = blockIdx.x;
  const int64_t b = blockIdx.y;
  const int64_t row = sets[b * kSetFields + kSetRow];
  const int64_t nt = sets[b * kSetFields + kSetTiles];
  double s = 0.0;
  for (int64_t t = threadIdx.x; t < nt; t += 256) s += partials[(row + t) * nraw + e];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) raw[b * nraw + e] = red[0];
}

__global__ void batch_combine_kernel(int nsets, const int64_t* __restrict__ sets, int p, int P,
                                     int nraw, int nout, const double* __restrict__ raw,
                                     double* __restrict__ out, int32_t* __restrict__ status) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nsets)
    combine_one(sets[(int64_t)b * kSetFields + kSetN], p, P, raw + (int64_t)b * nraw,
                out + (int64_t)b * nout, status + 2 * b);
}

__global__ void batch_fisher_kernel(int nsets, int P, int nout, const double* __restrict__ out,
                                    double* __restrict__ covparms, int32_t* __restrict__ status,
                                    double max_step) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nsets)
    fisher_one<kMaxParms>(P, out + (int64_t)b * nout, covparms + (int64_t)b * P, status + 2 * b,
                          max_step);
}

__global__ void fill_u32_kernel(unsigned int* __restrict__ x, int count, unsigned int v) {
  for (int e = threadIdx.x; e < count; e += blockDim.x) x[e] = v;
}

__global__ void batch_status_clear_kernel(int32_t* status, int nsets) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nsets) {
    status[2 * b] = 0;
    status[2 * b + 1] = INT32_MAX;
  }
}

// Loglik at the given beta and the scaled gradient from the adjoint sums
// (logdet, r'S r, grad[P]).
__global__ void adjoint_finalize_kernel(int64_t n, int P, const double* __restrict__ raw,
                                        const double* __restrict__ grad_out,
                                        double* __restrict__ loglik, double* __restrict__ dcovparms,
                                        int32_t* __restrict__ status) {
  if (threadIdx.x != 0) return;
  const double ll = -0.5 * ((double)n * log(2.0 * M_PI) + raw[0] + raw[1]);
  const double go = grad_out ? grad_out[0] : 1.0;
  bool finite = __builtin_isfinite(ll);
  for (int j = 0; j < P; ++j) {
    dcovparms[j] = go * raw[2 + j];
    finite = finite && __builtin_isfinite(raw[2 + j]);
  }
  if (loglik) loglik[0] = ll;
  if (!finite) atomicOr(&status[0], VEC_FLAG_NONFINITE);
}

static int hip_code(hipError_t e) { return e == hipSuccess ? VEC_OK : VEC_EHIP; }

// Doubles per neighbourhood-sum vector of one kernel mode.
static int nraw_for(const Dims& dm, int mode) { return nraw_mode(mode, dm.p, dm.P); }

static int enqueue_block_sums(const vec_problem* pb, const Dims& dm, int mode, const double* locs,
                              const int32_t* NN, const double* y, const double* X,
                              const double* covparms, const double* beta, int64_t i0, int64_t i1,
                              double* partials, size_t partials_bytes, int* grid_out,
                              int32_t* status, hipStream_t st, double* rows_out = nullptr,
                              const int32_t* index = nullptr, int64_t nn_row0 = 0,
                              bool short_rows = false) {
  if (dm.wave) {
    // the sums of Algorithm 1 with their derivatives and information only
    if (mode != kModeSums || rows_out || index || nn_row0 != 0 || short_rows) return VEC_EINVAL;
    const int grid = vecchia_wave::wave_grid(i1 - i0);
    *grid_out = grid;
    if (grid == 0) return VEC_OK;
    if (!partials || partials_bytes < (size_t)grid * dm.nraw * sizeof(double))
      return VEC_EWORKSPACE;
    vecchia_wave::WaveArgs args = {};
    args.m = pb->m;
    args.d = pb->d;
    args.family = pb->family;
    args.nspace = pb->nspace;
    args.R = dm.P - 2;
    args.p = dm.p;
    args.nu = dm.nu;
    args.locs = locs;
    args.NN = NN;
    args.y = y;
    args.X = X;
    args.covparms = covparms;
    args.i0 = i0;
    args.i1 = i1;
    args.partials = partials;
    args.status = status;
    return hip_code(vecchia_wave::launch_wave(args, grid, st));
  }
  const int grid = grid_for(i1 - i0);
  *grid_out = grid;
  if (grid == 0) return VEC_OK;
  const size_t need = (size_t)grid * nraw_for(dm, mode) * sizeof(double);
  if (!partials || partials_bytes < need) return VEC_EWORKSPACE;
  const int pc = dm.p - 1, ng = (pb->family == VEC_FAMILY_SPACETIME) ? 1 : 0;
  SumsArgs args = {};
  args.m = pb->m;
  args.d = pb->d;
  args.nspace = pb->nspace;
  args.nu = dm.nu;
  args.locs = locs;
  args.NN = NN;
  args.y = y;
  args.X = X;
  args.covparms = covparms;
  args.beta = beta;
  args.i0 = i0;
  args.i1 = i1;
  args.partials = partials;
  args.status = status;
  args.rows_out = rows_out;
  args.index = index;
  args.n = pb->n;
  args.nn_row0 = nn_row0;
  args.short_rows = short_rows ? 1 : 0;
  return hip_code(kLaunch[dm.kidx][pc][ng][mode](grid, st, args));
}

// Kernel pass over [i0, i1) followed by the fixed-order reduction into raw.
static int enqueue_sums(const vec_problem* pb, const Dims& dm, int mode, const double* locs,
                        const int32_t* NN, const double* y, const double* X,
                        const double* covparms, const double* beta, int64_t i0, int64_t i1,
                        double* raw, void* workspace, size_t workspace_bytes, int32_t* status,
                        hipStream_t st, double* rows_out = nullptr,
                        const int32_t* index = nullptr,
                        int64_t nn_row0 = 0, bool short_rows = false) {
  const int64_t total = i1 - i0;
  const int nraw = nraw_for(dm, mode);
  if (total == 0) {
    hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(64), 0, st, raw, nraw, 0.0);
    return hip_code(hipGetLastError());
  }
  double* partials = static_cast<double*>(workspace);
  int grid = 0;
  int rc = enqueue_block_sums(pb, dm, mode, locs, NN, y, X, covparms, beta, i0, i1, partials,
                              workspace_bytes, &grid, status, st, rows_out, index, nn_row0,
                              short_rows);
  if (rc != VEC_OK) return rc;
  hipLaunchKernelGGL(reduce_kernel, dim3(nraw), dim3(256), 0, st, partials, grid, nraw, raw);
  return hip_code(hipGetLastError());
}

// ----------------------------------------------------------------------------
// batches of datasets
// ----------------------------------------------------------------------------

static_assert(VEC_NUM_CLASSES == kNumBatchK, "one size class per batched kernel size");
constexpr int kDefaultTile = 32;
constexpr int kMaxTile = 1 << 20;
constexpr int kMaxSets = 65535;

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Device plan layout: sets[nsets][kSetFields] int64, then per class the
// tile prefix [nsets + 1] int64, then per class the dataset ids [nsets] int32.
struct PlanLayout {
  size_t sets, prefix, ids, bytes;
};
static PlanLayout plan_layout(int32_t nsets) {
  PlanLayout L;
  L.sets = 0;
  L.prefix = align256((size_t)nsets * kSetFields * sizeof(int64_t));
  L.ids = L.prefix + align256((size_t)kNumBatchK * (nsets + 1) * sizeof(int64_t));
  L.bytes = L.ids + align256((size_t)kNumBatchK * nsets * sizeof(int32_t));
  return L;
}

static bool batch_dims(const vec_batch* bt, Dims* dm) {
  if (!bt || bt->nsets < 1 || bt->nsets > kMaxSets || bt->reserved != 0) return false;
  if (bt->n_total < 1 || bt->nn_total < 0) return false;
  vec_problem pb = {};
  pb.n = 1;
  pb.m = 0;
  pb.d = bt->d;
  pb.p = bt->p;
  pb.family = bt->family;
  pb.smoothness = 0.5;
  pb.nspace = bt->nspace;
  return dims_of(&pb, dm) && !dm->wave;
}

static int nu_code(double smoothness) {
  if (smoothness == 0.5) return 0;
  if (smoothness == 1.5) return 1;
  if (smoothness == 2.5) return 2;
  return -1;
}

static size_t batch_ws_bytes(const Dims& dm, const vec_batch_plan* plan) {
  return align256((size_t)plan->rows * dm.nraw * sizeof(double)) + 256;
}

static int enqueue_batch_sums(const vec_batch* bt, const Dims& dm, const vec_batch_plan* plan,
                              const void* plan_dev, const double* locs, const int32_t* NN,
                              const double* y, const double* X, const double* covparms,
                              double* raw, void* ws, int32_t* status, hipStream_t st) {
  const PlanLayout L = plan_layout(plan->nsets);
  const char* pd = static_cast<const char*>(plan_dev);
  double* partials = static_cast<double*>(ws);
  unsigned int* counters = reinterpret_cast<unsigned int*>(
      static_cast<char*>(ws) + align256((size_t)plan->rows * dm.nraw * sizeof(double)));
  hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, st, counters, kNumBatchK, 0u);
  const int pc = dm.p - 1, ng = (bt->family == VEC_FAMILY_SPACETIME) ? 1 : 0;
  int64_t row0 = 0;
  // largest neighbourhoods first
  for (int c = kNumBatchK - 1; c >= 0; --c) {
    if (plan->ntiles[c] == 0) continue;
    SumsArgs args = {};
    args.d = bt->d;
    args.nspace = bt->nspace;
    args.locs = locs;
    args.NN = NN;
    args.y = y;
    args.X = X;
    args.covparms = covparms;
    args.partials = partials;
    args.status = status;
    args.batch.sets = reinterpret_cast<const int64_t*>(pd + L.sets);
    args.batch.class_prefix = reinterpret_cast<const int64_t*>(pd + L.prefix) +
                              (size_t)c * (plan->nsets + 1);
    args.batch.class_sets = reinterpret_cast<const int32_t*>(pd + L.ids) + (size_t)c * plan->nsets;
    args.batch.counter = counters + c;
    args.batch.count = plan->count[c];
    args.batch.tile = plan->sched.tile[c];
    // class c's rows follow those of the classes below it
    row0 = 0;
    for (int k = 0; k < c; ++k) row0 += plan->ntiles[k];
    args.batch.row0 = row0;
    hipError_t e = kLaunchBatch[c][pc][ng](plan->grid[c], st, args);
    if (e != hipSuccess) return VEC_EHIP;
  }
  hipLaunchKernelGGL(batch_reduce_kernel, dim3(dm.nraw, plan->nsets), dim3(256), 0, st,
                     reinterpret_cast<const int64_t*>(pd + L.sets), partials, dm.nraw, raw);
  return hip_code(hipGetLastError());
}

static int check_batch_call(const vec_batch* bt, const vec_batch_plan* plan, const void* plan_dev,
                            const void* locs, const void* NN, const void* y, const void* X,
                            const void* covparms, const void* raw, void* ws, size_t wsb,
                            const void* status, Dims* dm) {
  if (!batch_dims(bt, dm) || !plan || plan->nsets != bt->nsets) return VEC_EINVAL;
  if (!plan_dev || !locs || !NN || !y || !X || !covparms || !raw || !status) return VEC_EINVAL;
  if (!ws || wsb < batch_ws_bytes(*dm, plan)) return VEC_EWORKSPACE;
  return VEC_OK;
}

// Grouped sums on the fused kernel.  A block's conditional density
// p(y_B | y_N) is the product of its members' one-observation conditionals,
// member k conditioned on N and on members 0..k-1 (the chain rule of the
// Gaussian density, exact), and the expected information of the block
// conditional is the sum of theirs (each factor's score has mean zero given
// everything the later factors condition on).  So the block's raw sums are
// those of ordinary neighbourhoods whose NNarray rows list N and the earlier
// members: row i of the expanded array (width m + max_block) holds i, the
// block's conditioning set, the members before i, then -1.  Rows of
// observations outside every block keep -1 in column 0 and are skipped.
__global__ void grouped_clear_rows_kernel(int64_t n, int width, int32_t* __restrict__ NN) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    NN[i * width] = -1;
}

// one wave per block: the block's rows are one contiguous span of the
// expanded array, written by consecutive lanes
__global__ __launch_bounds__(64) void grouped_expand_kernel(
    const int64_t* __restrict__ block_start, const int64_t* __restrict__ cond_start,
    const int32_t* __restrict__ cond, int64_t ncond, int m, int gmax, int64_t n, int width,
    int32_t* __restrict__ NN, int32_t* __restrict__ status) {
  const int64_t b = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t first = block_start[b], last = block_start[b + 1];
  const int64_t c0 = cond_start[b], c1 = cond_start[b + 1];
  const bool ok = first >= 0 && last > first && last - first <= gmax && last <= n && c0 >= 0 &&
                  c1 >= c0 && c1 <= ncond && c1 - c0 <= m;
  if (!ok) {
    if (lane == 0) {
      atomicOr(&status[0], VEC_FLAG_BADNN);
      atomicMin(&status[1], (int32_t)(first > 0 ? first : 0));
    }
    return;
  }
  // indices are earlier observations, at most `first` distinct ones
  bool bad = false;
  for (int64_t q = c0 + lane; q < c1; q += 64) bad = bad || cond[q] < 0 || (int64_t)cond[q] >= first;
  if (__ballot(bad) != 0ull || c1 - c0 > first) {
    if (lane == 0) {
      atomicOr(&status[0], VEC_FLAG_BADNN);
      atomicMin(&status[1], (int32_t)first);
    }
    return;
  }
  const int c = (int)(c1 - c0);
  const int64_t total = (last - first) * width;
  int32_t* span = NN + first * width;
  for (int64_t e = lane; e < total; e += 64) {
    const int k = (int)(e / width), col = (int)(e % width);
    int32_t v;
    if (col == 0)
      v = (int32_t)(first + k);
    else if (col <= c)
      v = cond[c0 + col - 1];
    else if (col <= c + k)
      v = (int32_t)(first + (col - 1 - c));
    else
      v = -1;
    span[e] = v;
  }
}

// The problem whose neighbourhoods are the expanded rows, if the fused
// kernel takes it (family and split it serves, m + max_block - 1 <= 60).
static bool grouped_fused_dims(const vec_problem* pb, int32_t max_block, vec_problem* q,
                               Dims* dq) {
  *q = *pb;
  q->m = pb->m + max_block - 1;
  return dims_of(q, dq) && !dq->wave;
}

static size_t grouped_fused_bytes(const vec_problem* q, const Dims& dq) {
  const int grid = grid_for(q->n);
  return align256((size_t)q->n * (q->m + 1) * sizeof(int32_t)) +
         (size_t)(grid > 0 ? grid : 1) * dq.nraw * sizeof(double);
}

// Grouped sums: the fused kernel over the expanded rows where it applies,
// else one wave per block; then the fixed-order reduction.  Fisher scoring
// expands the rows once (they do not depend on the parameters) and sums
// each iteration.
enum GroupedStep { kGroupedExpandAndSum = 0, kGroupedExpand = 1, kGroupedSum = 2 };

static int check_grouped(const vec_problem* pb, const Dims& dm, int64_t nblocks, int32_t max_block) {
  if (nblocks < 0 || max_block < 1 || max_block > vecchia_wave::kMaxBlock) return VEC_EINVAL;
  if (max_block > 1 && pb->d > 4) return VEC_EINVAL;
  if (pb->m + max_block > vecchia_wave::kMaxK) return VEC_EINVAL;
  if (1 + dm.p + (dm.P - 1) * max_block > 64) return VEC_EINVAL;  // solved columns
  return VEC_OK;
}

static int enqueue_grouped_sums(const vec_problem* pb, const Dims& dm, const double* locs,
                                const double* y, const double* X, const double* covparms,
                                int64_t nblocks, const int64_t* block_start,
                                const int64_t* cond_start, const int32_t* cond, int64_t ncond,
                                int32_t max_block, double* raw, void* workspace,
                                size_t workspace_bytes, int32_t* status, hipStream_t st,
                                GroupedStep step = kGroupedExpandAndSum) {
  if (nblocks == 0) {
    if (step == kGroupedExpand) return VEC_OK;
    hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(64), 0, st, raw, dm.nraw, 0.0);
    return hip_code(hipGetLastError());
  }
  vec_problem q;
  Dims dq;
  if (grouped_fused_dims(pb, max_block, &q, &dq)) {
    if (!workspace || workspace_bytes < grouped_fused_bytes(&q, dq)) return VEC_EWORKSPACE;
    const int width = q.m + 1;
    int32_t* NNx = static_cast<int32_t*>(workspace);
    const size_t nnb = align256((size_t)q.n * width * sizeof(int32_t));
    if (step != kGroupedSum) {
      hipLaunchKernelGGL(grouped_clear_rows_kernel, dim3(1024), dim3(256), 0, st, q.n, width, NNx);
      hipLaunchKernelGGL(grouped_expand_kernel, dim3((unsigned)nblocks), dim3(64), 0, st,
                         block_start, cond_start, cond, ncond, pb->m, max_block, q.n, width, NNx,
                         status);
      if (hipGetLastError() != hipSuccess) return VEC_EHIP;
      if (step == kGroupedExpand) return VEC_OK;
    }
    return enqueue_sums(&q, dq, kModeSums, locs, NNx, y, X, covparms, nullptr, 0, q.n, raw,
                        static_cast<char*>(workspace) + nnb, workspace_bytes - nnb, status, st,
                        nullptr, nullptr, 0, true);
  }
  if (step == kGroupedExpand) return VEC_OK;  // the wave kernel reads the blocks directly
  const int grid = vecchia_wave::wave_grid(nblocks);
  if (!workspace || workspace_bytes < (size_t)grid * dm.nraw * sizeof(double))
    return VEC_EWORKSPACE;
  vecchia_wave::WaveArgs args = {};
  args.m = pb->m;
  args.d = pb->d;
  args.p = dm.p;
  args.nu = dm.nu;
  args.family = pb->family;
  args.nspace = pb->nspace;
  args.R = dm.P - 2;
  args.locs = locs;
  args.y = y;
  args.X = X;
  args.covparms = covparms;
  args.i0 = 0;
  args.i1 = nblocks;
  args.block_start = block_start;
  args.cond_start = cond_start;
  args.cond = cond;
  args.ncond = ncond;
  args.gmax = max_block;
  args.n = pb->n;
  args.partials = static_cast<double*>(workspace);
  args.status = status;
  if (vecchia_wave::launch_wave(args, grid, st) != hipSuccess) return VEC_EHIP;
  hipLaunchKernelGGL(reduce_kernel, dim3(dm.nraw), dim3(256), 0, st, args.partials, grid, dm.nraw,
                     raw);
  return hip_code(hipGetLastError());
}

}  // namespace vecchia

using namespace vecchia;

// ----------------------------------------------------------------------------
// device scratch of the allocation-free entry point
// ----------------------------------------------------------------------------

// Partial sums of vecchia_loglik_grad_info_noalloc: one copy per device,
// held from the library's first use on that device until the process ends.
// Host code never names the array in a kernel argument or a copy: the name
// is a host-side stand-in; the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kScratchBytes = (size_t)2 << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device.
static int scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return VEC_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return VEC_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return VEC_EHIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return VEC_OK;
}

extern "C" {

int vec_nparms(const vec_problem* pb) {
  Dims dm;
  return dims_of(pb, &dm) ? dm.P : VEC_EINVAL;
}

int vec_nraw(const vec_problem* pb) {
  Dims dm;
  return dims_of(pb, &dm) ? dm.nraw : VEC_EINVAL;
}

int vec_nout(const vec_problem* pb) {
  Dims dm;
  return dims_of(pb, &dm) ? dm.nout : VEC_EINVAL;
}

int vec_max_m(void) { return kKs[kNumK - 1] - 1; }

size_t vec_workspace_bytes(const vec_problem* pb, int64_t i0, int64_t i1) {
  Dims dm;
  if (!dims_of(pb, &dm) || i0 < 0 || i1 < i0 || i1 > pb->n) return 0;
  const int grid = dm.wave ? vecchia_wave::wave_grid(i1 - i0) : grid_for(i1 - i0);
  return (size_t)(grid > 0 ? grid : 1) * dm.nraw * sizeof(double);
}

int vec_raw_sums(const vec_problem* pb, const double* locs, const int32_t* NNarray,
                 const double* y, const double* X, const double* covparms, int64_t i0,
                 int64_t i1, double* raw, void* workspace, size_t workspace_bytes,
                 int32_t* status, void* stream) {
  Dims dm;
  if (!dims_of(pb, &dm)) return VEC_EINVAL;
  if (i0 < 0 || i1 < i0 || i1 > pb->n) return VEC_EINVAL;
  if (!locs || !NNarray || !y || !X || !covparms || !raw || !status) return VEC_EINVAL;
  return enqueue_sums(pb, dm, kModeSums, locs, NNarray, y, X, covparms, nullptr, i0, i1, raw,
                      workspace, workspace_bytes, status, static_cast<hipStream_t>(stream));
}

int vec_block_sums(const vec_problem* pb, const double* locs, const int32_t* NNarray,
                   const double* y, const double* X, const double* covparms, int64_t i0,
                   int64_t i1, double* partials, size_t partials_bytes, int32_t* nblocks,
                   int32_t* status, void* stream) {
  Dims dm;
  if (!dims_of(pb, &dm) || !nblocks) return VEC_EINVAL;
  if (i0 < 0 || i1 < i0 || i1 > pb->n) return VEC_EINVAL;
  if (!locs || !NNarray || !y || !X || !covparms || !status) return VEC_EINVAL;
  int grid = 0;
  int rc = enqueue_block_sums(pb, dm, kModeSums, locs, NNarray, y, X, covparms, nullptr, i0, i1,
                              partials, partials_bytes, &grid, status,
                              static_cast<hipStream_t>(stream));
  *nblocks = grid;
  return rc;
}

int vec_combine(const vec_problem* pb, const double* raw, double* out, int32_t* status,
                void* stream) {
  Dims dm;
  if (!dims_of(pb, &dm) || !raw || !out || !status) return VEC_EINVAL;
  enqueue_combine(pb, dm, raw, out, status, static_cast<hipStream_t>(stream));
  return hip_code(hipGetLastError());
}

int vecchia_loglik_grad_info(const vec_problem* pb, const double* locs, const int32_t* NNarray,
                         const double* y, const double* X, const double* covparms, double* raw,
                         double* out, void* workspace, size_t workspace_bytes, int32_t* status,
                         void* stream) {
  int rc = vec_raw_sums(pb, locs, NNarray, y, X, covparms, 0, pb ? pb->n : 0, raw, workspace,
                        workspace_bytes, status, stream);
  if (rc != VEC_OK) return rc;
  return vec_combine(pb, raw, out, status, stream);
}

int vecchia_loglik_grad_info_noalloc(const vec_problem* pb, const double* locs,
                                     const int32_t* NNarray, const double* y, const double* X,
                                     const double* covparms, double* raw, double* out,
                                     int32_t* status, void* stream) {
  Dims dm;
  if (!dims_of(pb, &dm)) return VEC_EINVAL;
  if (!locs || !NNarray || !y || !X || !covparms || !raw || !out || !status) return VEC_EINVAL;
  // every workgroup writes its whole row of partials, so nothing in the
  // scratch array has to start at zero
  const size_t need = vec_workspace_bytes(pb, 0, pb->n);
  if (need > kScratchBytes) return VEC_EWORKSPACE;
  void* ws = nullptr;
  const int rc = scratch_address(&ws);
  if (rc != VEC_OK) return rc;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const int rs = enqueue_sums(pb, dm, kModeSums, locs, NNarray, y, X, covparms, nullptr, 0, pb->n,
                              raw, ws, kScratchBytes, status, st);
  if (rs != VEC_OK) return rs;
  enqueue_combine(pb, dm, raw, out, status, st);
  return hip_code(hipGetLastError());
}

int vec_loglik(const vec_problem* pb, const double* locs, const int32_t* NNarray, const double* y,
               const double* X, const double* covparms, double* raw, double* out, void* workspace,
               size_t workspace_bytes, int32_t* status, void* stream) {
  Dims dm;
  if (!dims_of(pb, &dm)) return VEC_EINVAL;
  if (!locs || !NNarray || !y || !X || !covparms || !raw || !out || !status) return VEC_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = enqueue_sums(pb, dm, kModeLoglik, locs, NNarray, y, X, covparms, nullptr, 0, pb->n, raw,
                        workspace, workspace_bytes, status, st);
  if (rc != VEC_OK) return rc;
  // the combine step with no covariance parameters: loglik, betahat, betainfo
  hipLaunchKernelGGL(combine_kernel, dim3(1), dim3(64), 0, st, pb->n, dm.p, 0, raw, out, status);
  return hip_code(hipGetLastError());
}

int vec_loglik_adjoint(const vec_problem* pb, const double* locs, const int32_t* NNarray,
                       const double* y, const double* X, const double* covparms,
                       const double* betahat, const double* grad_out, double* loglik,
                       double* dcovparms, void* workspace, size_t workspace_bytes,
                       int32_t* status, void* stream) {
  Dims dm;
  if (!dims_of(pb, &dm)) return VEC_EINVAL;
  if (!locs || !NNarray || !y || !X || !covparms || !betahat || !dcovparms || !status)
    return VEC_EINVAL;
  if (!workspace) return VEC_EWORKSPACE;
  // partials first, the reduced vector (2 + P doubles) at the end
  const int nraw = nraw_for(dm, kModeAdjoint);
  const int grid = grid_for(pb->n);
  const size_t part_bytes = (size_t)grid * nraw * sizeof(double);
  if (workspace_bytes < part_bytes + nraw * sizeof(double)) return VEC_EWORKSPACE;
  double* raw = reinterpret_cast<double*>(static_cast<char*>(workspace) + part_bytes);
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = enqueue_sums(pb, dm, kModeAdjoint, locs, NNarray, y, X, covparms, betahat, 0, pb->n,
                        raw, workspace, part_bytes, status, st);
  if (rc != VEC_OK) return rc;
  hipLaunchKernelGGL(adjoint_finalize_kernel, dim3(1), dim3(64), 0, st, pb->n, dm.P, raw,
                     grad_out, loglik, dcovparms, status);
  return hip_code(hipGetLastError());
}

int vec_kriging_weights(const vec_problem* pb, const double* locs, const int32_t* NNarray,
                        const double* y, const double* X, const double* covparms, int64_t i0,
                        int64_t i1, double* weights, double* raw, void* workspace,
                        size_t workspace_bytes, int32_t* status, void* stream) {
  Dims dm;
  if (!dims_of(pb, &dm)) return VEC_EINVAL;
  if (i0 < 0 || i1 < i0 || i1 > pb->n) return VEC_EINVAL;
  if (!locs || !NNarray || !y || !X || !covparms || !weights || !raw || !status)
    return VEC_EINVAL;
  return enqueue_sums(pb, dm, kModeWeights, locs, NNarray, y, X, covparms, nullptr, i0, i1, raw,
                      workspace, workspace_bytes, status, static_cast<hipStream_t>(stream),
                      weights);
}

size_t vec_kriging_predict_workspace_bytes(const vec_problem* pb, int64_t n_obs) {
  Dims dm;
  if (!dims_of(pb, &dm) || dm.wave || n_obs < pb->m || n_obs >= pb->n) return 0;
  const int64_t n_pred = pb->n - n_obs;
  return align256(vec_workspace_bytes(pb, n_obs, pb->n)) +
         align256((size_t)n_pred * (pb->m + 1) * sizeof(double)) +
         align256((size_t)nraw_of(dm.p, 0) * sizeof(double));
}

int vec_kriging_predict(const vec_problem* pb, const double* locs, const int32_t* NN_pred,
                        const double* y, const double* X, const double* covparms,
                        const double* betahat, int64_t n_obs, double* mean, double* var,
                        void* workspace, size_t workspace_bytes, int32_t* status, void* stream) {
  Dims dm;
  if (!dims_of(pb, &dm) || dm.wave || n_obs < pb->m || n_obs >= pb->n) return VEC_EINVAL;
  if (!locs || !NN_pred || !y || !X || !covparms || !betahat || !mean || !var || !status)
    return VEC_EINVAL;
  const size_t need = vec_kriging_predict_workspace_bytes(pb, n_obs);
  if (!workspace || workspace_bytes < need) return VEC_EWORKSPACE;
  const int64_t n_pred = pb->n - n_obs;
  char* w = static_cast<char*>(workspace);
  const size_t part = align256(vec_workspace_bytes(pb, n_obs, pb->n));
  double* rows = reinterpret_cast<double*>(w + part);
  double* raw = reinterpret_cast<double*>(w + part + align256((size_t)n_pred * (pb->m + 1) * 8));
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = enqueue_sums(pb, dm, kModeWeights, locs, NN_pred, y, X, covparms, nullptr, n_obs, pb->n,
                        raw, workspace, part, status, st, rows, nullptr, n_obs);
  if (rc != VEC_OK) return rc;
  hipLaunchKernelGGL(predict_kernel, dim3((unsigned)((n_pred + 255) / 256)), dim3(256), 0, st, n_obs,
                     n_pred, pb->m, dm.p, NN_pred, y, X, betahat, covparms, rows, mean, var);
  return hip_code(hipGetLastError());
}

int vec_combine_loglik(const vec_problem* pb, const double* raw_a, const double* raw_b,
                       double* raw_sum, double* out, int32_t* status, void* stream) {
  Dims dm;
  if (!dims_of(pb, &dm) || !raw_a || !raw_sum || !out || !status) return VEC_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(add_raw_kernel, dim3(1), dim3(64), 0, st, raw_a, raw_b, nraw_of(dm.p, 0),
                     raw_sum);
  hipLaunchKernelGGL(combine_kernel, dim3(1), dim3(64), 0, st, pb->n, dm.p, 0, raw_sum, out, status);
  return hip_code(hipGetLastError());
}

int vec_loglik_sums_at(const vec_problem* pb, const double* locs, const int32_t* NNarray,
                       const double* y, const double* X, const double* covparms,
                       const int32_t* index, int64_t count, double* raw, void* workspace,
                       size_t workspace_bytes, int32_t* status, void* stream) {
  Dims dm;
  if (!dims_of(pb, &dm) || count < 0 || count > pb->n) return VEC_EINVAL;
  if (!locs || !NNarray || !y || !X || !covparms || !raw || !status) return VEC_EINVAL;
  if (count > 0 && !index) return VEC_EINVAL;
  return enqueue_sums(pb, dm, kModeLoglik, locs, NNarray, y, X, covparms, nullptr, 0, count, raw,
                      workspace, workspace_bytes, status, static_cast<hipStream_t>(stream),
                      nullptr, index);
}

int vec_fisher_update(const vec_problem* pb, const double* out, double* covparms,
                      int32_t* status, double max_step, void* stream) {
  Dims dm;
  if (!dims_of(pb, &dm) || !out || !covparms || !status || !(max_step > 0.0)) return VEC_EINVAL;
  enqueue_fisher(dm, out, covparms, status, max_step, static_cast<hipStream_t>(stream));
  return hip_code(hipGetLastError());
}

int vec_status_clear(int32_t* status, void* stream) {
  if (!status) return VEC_EINVAL;
  hipLaunchKernelGGL(status_clear_kernel, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream),
                     status);
  return hip_code(hipGetLastError());
}

int vec_status_code(const int32_t* host_status) {
  if (!host_status) return VEC_EINVAL;
  const int f = host_status[0];
  if (f & VEC_FLAG_BADNN) return VEC_EBADNN;
  if (f & VEC_FLAG_NOTPD) return VEC_ENOTPD;
  if (f & VEC_FLAG_NONFINITE) return VEC_ENONFINITE;
  return VEC_OK;
}

static int one_iteration(const vec_problem* pb, const Dims& dm, const double* locs,
                         const int32_t* NN, const double* y, const double* X, double* covparms,
                         double max_step, double* raw, double* out, void* ws, size_t wsb,
                         int32_t* status, hipStream_t st) {
  int rc = enqueue_sums(pb, dm, kModeSums, locs, NN, y, X, covparms, nullptr, 0, pb->n, raw, ws,
                        wsb, status, st);
  if (rc != VEC_OK) return rc;
  enqueue_combine(pb, dm, raw, out, status, st);
  enqueue_fisher(dm, out, covparms, status, max_step, st);
  return hip_code(hipGetLastError());
}

int vec_fisher_fit(const vec_problem* pb, const double* locs, const int32_t* NNarray,
                   const double* y, const double* X, double* covparms, int32_t iters,
                   double max_step, double* raw, double* out, void* workspace,
                   size_t workspace_bytes, int32_t* status, int32_t use_graph, void* stream) {
  Dims dm;
  if (!dims_of(pb, &dm) || iters < 0 || !(max_step > 0.0)) return VEC_EINVAL;
  if (!locs || !NNarray || !y || !X || !covparms || !raw || !out || !status) return VEC_EINVAL;
  if (workspace_bytes < vec_workspace_bytes(pb, 0, pb->n) || !workspace) return VEC_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!use_graph || st == nullptr || iters == 0) {
    for (int it = 0; it < iters; ++it) {
      int rc = one_iteration(pb, dm, locs, NNarray, y, X, covparms, max_step, raw, out, workspace,
                             workspace_bytes, status, st);
      if (rc != VEC_OK) return rc;
    }
    return VEC_OK;
  }
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return VEC_EHIP;
  int rc = one_iteration(pb, dm, locs, NNarray, y, X, covparms, max_step, raw, out, workspace,
                         workspace_bytes, status, st);
  hipError_t e = hipStreamEndCapture(st, &graph);
  if (rc != VEC_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc != VEC_OK ? rc : VEC_EHIP;
  }
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e == hipSuccess) {
    for (int it = 0; it < iters && e == hipSuccess; ++it) e = hipGraphLaunch(exec, st);
    (void)hipGraphExecDestroy(exec);
  }
  (void)hipGraphDestroy(graph);
  return hip_code(e);
}

size_t vec_grouped_workspace_bytes(const vec_problem* pb, int64_t nblocks) {
  Dims dm;
  if (!dims_of(pb, &dm) || nblocks < 0) return 0;
  const int grid = vecchia_wave::wave_grid(nblocks);
  size_t bytes = (size_t)(grid > 0 ? grid : 1) * dm.nraw * sizeof(double);
  // the fused route for any block size it serves
  for (int32_t g = 1; g <= vecchia_wave::kMaxBlock; ++g) {
    vec_problem q;
    Dims dq;
    if (grouped_fused_dims(pb, g, &q, &dq)) bytes = std::max(bytes, grouped_fused_bytes(&q, dq));
  }
  return bytes;
}

int vec_grouped_raw_sums(const vec_problem* pb, const double* locs, const double* y,
                         const double* X, const double* covparms, int64_t nblocks,
                         const int64_t* block_start, const int64_t* cond_start,
                         const int32_t* cond, int64_t ncond, int32_t max_block, double* raw,
                         void* workspace, size_t workspace_bytes, int32_t* status, void* stream) {
  Dims dm;
  if (!dims_of(pb, &dm)) return VEC_EINVAL;
  int rc = check_grouped(pb, dm, nblocks, max_block);
  if (rc != VEC_OK) return rc;
  if (!locs || !y || !X || !covparms || !raw || !status || ncond < 0) return VEC_EINVAL;
  if (nblocks > 0 && (!block_start || !cond_start || (ncond > 0 && !cond))) return VEC_EINVAL;
  return enqueue_grouped_sums(pb, dm, locs, y, X, covparms, nblocks, block_start, cond_start, cond,
                              ncond, max_block, raw, workspace, workspace_bytes, status,
                              static_cast<hipStream_t>(stream));
}

int vec_grouped_fisher_fit(const vec_problem* pb, const double* locs, const double* y,
                           const double* X, double* covparms, int64_t nblocks,
                           const int64_t* block_start, const int64_t* cond_start,
                           const int32_t* cond, int64_t ncond, int32_t max_block, int32_t iters,
                           double max_step, double* raw, double* out, void* workspace,
                           size_t workspace_bytes, int32_t* status, int32_t use_graph,
                           void* stream) {
  Dims dm;
  if (!dims_of(pb, &dm) || iters < 0 || !(max_step > 0.0)) return VEC_EINVAL;
  int rc = check_grouped(pb, dm, nblocks, max_block);
  if (rc != VEC_OK) return rc;
  if (!locs || !y || !X || !covparms || !raw || !out || !status || ncond < 0) return VEC_EINVAL;
  if (nblocks > 0 && (!block_start || !cond_start || (ncond > 0 && !cond))) return VEC_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (iters > 0) {
    rc = enqueue_grouped_sums(pb, dm, locs, y, X, covparms, nblocks, block_start, cond_start, cond,
                              ncond, max_block, raw, workspace, workspace_bytes, status, st,
                              kGroupedExpand);
    if (rc != VEC_OK) return rc;
  }
  auto one = [&]() -> int {
    int r = enqueue_grouped_sums(pb, dm, locs, y, X, covparms, nblocks, block_start, cond_start,
                                 cond, ncond, max_block, raw, workspace, workspace_bytes, status,
                                 st, kGroupedSum);
    if (r != VEC_OK) return r;
    enqueue_combine(pb, dm, raw, out, status, st);
    enqueue_fisher(dm, out, covparms, status, max_step, st);
    return hip_code(hipGetLastError());
  };
  if (!use_graph || st == nullptr || iters == 0) {
    for (int it = 0; it < iters; ++it) {
      rc = one();
      if (rc != VEC_OK) return rc;
    }
    return VEC_OK;
  }
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return VEC_EHIP;
  rc = one();
  hipError_t e = hipStreamEndCapture(st, &graph);
  if (rc != VEC_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc != VEC_OK ? rc : VEC_EHIP;
  }
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e == hipSuccess) {
    for (int it = 0; it < iters && e == hipSuccess; ++it) e = hipGraphLaunch(exec, st);
    (void)hipGraphExecDestroy(exec);
  }
  (void)hipGraphDestroy(graph);
  return hip_code(e);
}

size_t vec_batch_plan_bytes(int32_t nsets) {
  if (nsets < 1 || nsets > kMaxSets) return 0;
  return plan_layout(nsets).bytes;
}

int vec_batch_make_plan(const vec_batch* bt, const vec_dataset* sets, const vec_schedule* sched,
                        vec_batch_plan* plan, void* plan_dev, size_t plan_dev_bytes,
                        void* stream) {
  Dims dm;
  if (!batch_dims(bt, &dm) || !sets || !plan || !plan_dev) return VEC_EINVAL;
  const int32_t ns = bt->nsets;
  const PlanLayout L = plan_layout(ns);
  if (plan_dev_bytes < L.bytes) return VEC_EWORKSPACE;
  vec_batch_plan pl = {};
  pl.nsets = ns;
  for (int c = 0; c < kNumBatchK; ++c) {
    const int t = sched ? sched->tile[c] : 0;
    const int b = sched ? sched->blocks_per_cu[c] : 0;
    if (t < 0 || t > kMaxTile || b < 0 || b > 64) return VEC_EINVAL;
    pl.sched.tile[c] = t ? t : kDefaultTile;
    pl.sched.blocks_per_cu[c] = b;
  }
  // validate every descriptor and find its class
  std::vector<int> cls(ns);
  for (int32_t b = 0; b < ns; ++b) {
    const vec_dataset& s = sets[b];
    if (s.reserved != 0 || s.n < 1 || s.n >= (int64_t)INT32_MAX) return VEC_EINVAL;
    if (s.m < 0 || s.m > kBatchKs[kNumBatchK - 1] - 1 || nu_code(s.smoothness) < 0) return VEC_EINVAL;
    if (s.obs_offset < 0 || s.obs_offset > bt->n_total - s.n) return VEC_EINVAL;
    const int64_t nn_entries = s.n * (int64_t)(s.m + 1);
    if (s.nn_offset < 0 || s.nn_offset > bt->nn_total - nn_entries) return VEC_EINVAL;
    int c = 0;
    while (s.m + 1 > kBatchKs[c]) ++c;
    cls[b] = c;
  }
  std::vector<int64_t> hsets((size_t)ns * kSetFields);
  std::vector<int64_t> hprefix((size_t)kNumBatchK * (ns + 1), 0);
  std::vector<int32_t> hids((size_t)kNumBatchK * ns, 0);
  int64_t row = 0;
  for (int c = 0; c < kNumBatchK; ++c) {
    int32_t cnt = 0;
    int64_t tiles = 0;
    int64_t* prefix = hprefix.data() + (size_t)c * (ns + 1);
    for (int32_t b = 0; b < ns; ++b) {
      if (cls[b] != c) continue;
      const vec_dataset& s = sets[b];
      const int64_t nt = (s.n + pl.sched.tile[c] - 1) / pl.sched.tile[c];
      int64_t* f = hsets.data() + (size_t)b * kSetFields;
      f[kSetObs] = s.obs_offset;
      f[kSetNN] = s.nn_offset;
      f[kSetN] = s.n;
      f[kSetM] = s.m;
      f[kSetNu] = nu_code(s.smoothness);
      f[kSetClass] = c;
      f[kSetRow] = row + tiles;
      f[kSetTiles] = nt;
      hids[(size_t)c * ns + cnt] = b;
      prefix[cnt] = tiles;
      tiles += nt;
      ++cnt;
    }
    prefix[cnt] = tiles;
    pl.count[c] = cnt;
    pl.ntiles[c] = tiles;
    row += tiles;
  }
  pl.rows = row;
  pl.plan_bytes = (int64_t)L.bytes;
  // persistent grid: resident workgroups per CU (or the schedule's), capped by the tiles
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      ncu = v;
  }
  const int pc = dm.p - 1, ng = (bt->family == VEC_FAMILY_SPACETIME) ? 1 : 0;
  for (int c = 0; c < kNumBatchK; ++c) {
    int per_cu = pl.sched.blocks_per_cu[c];
    if (per_cu == 0) per_cu = kResidentBatch[c][pc][ng]();
    if (per_cu <= 0) per_cu = 1;
    const int64_t g = (int64_t)ncu * per_cu;
    pl.grid[c] = (int32_t)(g < pl.ntiles[c] ? g : pl.ntiles[c]);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* pd = static_cast<char*>(plan_dev);
  if (hipMemcpyAsync(pd + L.sets, hsets.data(), hsets.size() * sizeof(int64_t),
                     hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(pd + L.prefix, hprefix.data(), hprefix.size() * sizeof(int64_t),
                     hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(pd + L.ids, hids.data(), hids.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return VEC_EHIP;
  *plan = pl;
  return VEC_OK;
}

size_t vec_batch_workspace_bytes(const vec_batch* bt, const vec_batch_plan* plan) {
  Dims dm;
  if (!batch_dims(bt, &dm) || !plan || plan->nsets != bt->nsets) return 0;
  return batch_ws_bytes(dm, plan);
}

int vec_batch_raw_sums(const vec_batch* bt, const vec_batch_plan* plan, const void* plan_dev,
                       const double* locs, const int32_t* NNarray, const double* y,
                       const double* X, const double* covparms, double* raw, void* workspace,
                       size_t workspace_bytes, int32_t* status, void* stream) {
  Dims dm;
  int rc = check_batch_call(bt, plan, plan_dev, locs, NNarray, y, X, covparms, raw, workspace,
                            workspace_bytes, status, &dm);
  if (rc != VEC_OK) return rc;
  return enqueue_batch_sums(bt, dm, plan, plan_dev, locs, NNarray, y, X, covparms, raw, workspace,
                            status, static_cast<hipStream_t>(stream));
}

static int batch_iteration(const vec_batch* bt, const Dims& dm, const vec_batch_plan* plan,
                           const void* plan_dev, const double* locs, const int32_t* NN,
                           const double* y, const double* X, double* covparms, double* raw,
                           double* out, void* ws, int32_t* status, bool update, double max_step,
                           hipStream_t st) {
  int rc = enqueue_batch_sums(bt, dm, plan, plan_dev, locs, NN, y, X, covparms, raw, ws, status, st);
  if (rc != VEC_OK) return rc;
  const PlanLayout L = plan_layout(plan->nsets);
  const int64_t* sets = reinterpret_cast<const int64_t*>(static_cast<const char*>(plan_dev) + L.sets);
  const int nb = (plan->nsets + 63) / 64;
  hipLaunchKernelGGL(batch_combine_kernel, dim3(nb), dim3(64), 0, st, plan->nsets, sets, dm.p,
                     dm.P, dm.nraw, dm.nout, raw, out, status);
  if (update)
    hipLaunchKernelGGL(batch_fisher_kernel, dim3(nb), dim3(64), 0, st, plan->nsets, dm.P, dm.nout,
                       out, covparms, status, max_step);
  return hip_code(hipGetLastError());
}

int vec_batch_loglik_grad_info(const vec_batch* bt, const vec_batch_plan* plan,
                               const void* plan_dev, const double* locs, const int32_t* NNarray,
                               const double* y, const double* X, const double* covparms,
                               double* raw, double* out, void* workspace, size_t workspace_bytes,
                               int32_t* status, void* stream) {
  Dims dm;
  int rc = check_batch_call(bt, plan, plan_dev, locs, NNarray, y, X, covparms, raw, workspace,
                            workspace_bytes, status, &dm);
  if (rc != VEC_OK) return rc;
  if (!out) return VEC_EINVAL;
  return batch_iteration(bt, dm, plan, plan_dev, locs, NNarray, y, X,
                         const_cast<double*>(covparms), raw, out, workspace, status, false, 1.0,
                         static_cast<hipStream_t>(stream));
}

int vec_batch_fisher_fit(const vec_batch* bt, const vec_batch_plan* plan, const void* plan_dev,
                         const double* locs, const int32_t* NNarray, const double* y,
                         const double* X, double* covparms, int32_t iters, double max_step,
                         double* raw, double* out, void* workspace, size_t workspace_bytes,
                         int32_t* status, int32_t use_graph, void* stream) {
  Dims dm;
  int rc = check_batch_call(bt, plan, plan_dev, locs, NNarray, y, X, covparms, raw, workspace,
                            workspace_bytes, status, &dm);
  if (rc != VEC_OK) return rc;
  if (!out || iters < 0 || !(max_step > 0.0)) return VEC_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!use_graph || st == nullptr || iters == 0) {
    for (int it = 0; it < iters; ++it) {
      rc = batch_iteration(bt, dm, plan, plan_dev, locs, NNarray, y, X, covparms, raw, out,
                           workspace, status, true, max_step, st);
      if (rc != VEC_OK) return rc;
    }
    return VEC_OK;
  }
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return VEC_EHIP;
  rc = batch_iteration(bt, dm, plan, plan_dev, locs, NNarray, y, X, covparms, raw, out, workspace,
                       status, true, max_step, st);
  hipError_t e = hipStreamEndCapture(st, &graph);
  if (rc != VEC_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc != VEC_OK ? rc : VEC_EHIP;
  }
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e == hipSuccess) {
    for (int it = 0; it < iters && e == hipSuccess; ++it) e = hipGraphLaunch(exec, st);
    (void)hipGraphExecDestroy(exec);
  }
  (void)hipGraphDestroy(graph);
  return hip_code(e);
}

int vec_batch_status_clear(int32_t* status, int32_t nsets, void* stream) {
  if (!status || nsets < 1 || nsets > kMaxSets) return VEC_EINVAL;
  hipLaunchKernelGGL(batch_status_clear_kernel, dim3((nsets + 63) / 64), dim3(64), 0,
                     static_cast<hipStream_t>(stream), status, nsets);
  return hip_code(hipGetLastError());
}

#ifdef VECCHIA_SECTION_TIMING
// Profiling build only: copy out and reset the per-section cycle counters.
int vec_debug_section_cycles(unsigned long long* host_out, int n) {
  if (n > kSections) n = kSections;
  if (hipMemcpyFromSymbol(host_out, HIP_SYMBOL(section_cycles), n * sizeof(unsigned long long)) !=
      hipSuccess)
    return VEC_EHIP;
  unsigned long long zero[kSections] = {};
  return hip_code(hipMemcpyToSymbol(HIP_SYMBOL(section_cycles), zero, sizeof(zero)));
}
#endif

}  // extern "C"

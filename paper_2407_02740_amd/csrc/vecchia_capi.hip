// C ABI of the Vecchia library (declarations and contract in vecchia.h) and
// the small single-workgroup kernels around the fused per-neighbourhood
// kernel: the fixed-order reduction of workgroup partials, the combine step
// ("separate function", Section 3), the Fisher-scoring update (Eq. 4) and
// the status word.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "vecchia.h"
#include "vecchia_kernels.hpp"

namespace vecchia {

#ifdef VECCHIA_SECTION_TIMING
__device__ unsigned long long section_cycles[kSections];
#endif

// Instantiations live in vecchia_inst_k*.hip (compiled in parallel).
#define VEC_DECLARE(K, PC, NG, MODE) extern template VECCHIA_LAUNCH_SIG(K, PC, NG, MODE)
#define VEC_DECLARE_K(K)                   \
  VECCHIA_FOR_MODES(VEC_DECLARE, K, 1);    \
  VECCHIA_FOR_MODES(VEC_DECLARE, K, 2);    \
  VECCHIA_FOR_MODES(VEC_DECLARE, K, 3)
VEC_DECLARE_K(11);
VEC_DECLARE_K(21);
VEC_DECLARE_K(31);

// kLaunch[K index][p - 1][space-time][mode]
#define VEC_NG(K, PC, NG) \
  {launch_sums<K, PC, NG, kModeSums>, launch_sums<K, PC, NG, kModeAdjoint>, launch_sums<K, PC, NG, kModeLoglik>}
#define VEC_PC(K, PC) {VEC_NG(K, PC, 1), VEC_NG(K, PC, 2)}
#define VEC_ROW(K) {VEC_PC(K, 1), VEC_PC(K, 2), VEC_PC(K, 3)}
static const launch_fn kLaunch[kNumK][3][2][3] = {VEC_ROW(11), VEC_ROW(21), VEC_ROW(31)};

constexpr int kBlocksPerCU = 8;
constexpr int kMaxP = 3;
constexpr int kMaxParms = 4;

struct Dims {
  int p, P, nraw, nout, kidx, nu;
};

static bool dims_of(const vec_problem* pb, Dims* dm) {
  if (!pb) return false;
  if (pb->n < 1 || pb->n >= (int64_t)INT32_MAX) return false;
  if (pb->m < 0 || pb->d < 1 || pb->d > 4 || pb->p < 1 || pb->p > kMaxP) return false;
  if (pb->reserved != 0) return false;
  if (pb->family == VEC_FAMILY_ISO) {
    dm->P = 3;
  } else if (pb->family == VEC_FAMILY_SPACETIME) {
    if (pb->nspace < 1 || pb->nspace >= pb->d) return false;
    dm->P = 4;
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
  if (dm->kidx < 0) return false;
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
__global__ void combine_kernel(int64_t n, int p, int P, const double* __restrict__ raw,
                               double* __restrict__ out, int32_t* __restrict__ status) {
  if (threadIdx.x != 0) return;
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

// Eq. (4) on the log scale with a step-length cap.
__global__ void fisher_kernel(int P, int p, const double* __restrict__ out,
                              double* __restrict__ covparms, int32_t* __restrict__ status,
                              double max_step) {
  if (threadIdx.x != 0) return;
  if (status[0] != 0) return;
  const double* grad = out + 1;
  const double* info = grad + P;
  double th[kMaxParms], g[kMaxParms], I[kMaxParms * kMaxParms];
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
                              int32_t* status, hipStream_t st) {
  const int grid = grid_for(i1 - i0);
  *grid_out = grid;
  if (grid == 0) return VEC_OK;
  const size_t need = (size_t)grid * nraw_for(dm, mode) * sizeof(double);
  if (!partials || partials_bytes < need) return VEC_EWORKSPACE;
  const int pc = dm.p - 1, ng = (pb->family == VEC_FAMILY_SPACETIME) ? 1 : 0;
  hipError_t e = kLaunch[dm.kidx][pc][ng][mode](grid, st, pb->m, pb->d, pb->nspace, dm.nu, locs,
                                                NN, y, X, covparms, beta, i0, i1, partials, status);
  return hip_code(e);
}

// Kernel pass over [i0, i1) followed by the fixed-order reduction into raw.
static int enqueue_sums(const vec_problem* pb, const Dims& dm, int mode, const double* locs,
                        const int32_t* NN, const double* y, const double* X,
                        const double* covparms, const double* beta, int64_t i0, int64_t i1,
                        double* raw, void* workspace, size_t workspace_bytes, int32_t* status,
                        hipStream_t st) {
  const int64_t total = i1 - i0;
  const int nraw = nraw_for(dm, mode);
  if (total == 0) {
    hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(64), 0, st, raw, nraw, 0.0);
    return hip_code(hipGetLastError());
  }
  double* partials = static_cast<double*>(workspace);
  int grid = 0;
  int rc = enqueue_block_sums(pb, dm, mode, locs, NN, y, X, covparms, beta, i0, i1, partials,
                              workspace_bytes, &grid, status, st);
  if (rc != VEC_OK) return rc;
  hipLaunchKernelGGL(reduce_kernel, dim3(nraw), dim3(256), 0, st, partials, grid, nraw, raw);
  return hip_code(hipGetLastError());
}

}  // namespace vecchia

using namespace vecchia;

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
  const int grid = grid_for(i1 - i0);
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
  hipLaunchKernelGGL(combine_kernel, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream), pb->n,
                     dm.p, dm.P, raw, out, status);
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

int vec_fisher_update(const vec_problem* pb, const double* out, double* covparms,
                      int32_t* status, double max_step, void* stream) {
  Dims dm;
  if (!dims_of(pb, &dm) || !out || !covparms || !status || !(max_step > 0.0)) return VEC_EINVAL;
  hipLaunchKernelGGL(fisher_kernel, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream), dm.P,
                     dm.p, out, covparms, status, max_step);
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
  hipLaunchKernelGGL(combine_kernel, dim3(1), dim3(64), 0, st, pb->n, dm.p, dm.P, raw, out, status);
  hipLaunchKernelGGL(fisher_kernel, dim3(1), dim3(64), 0, st, dm.P, dm.p, out, covparms, status,
                     max_step);
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
    if (graph) hipGraphDestroy(graph);
    return rc != VEC_OK ? rc : VEC_EHIP;
  }
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e == hipSuccess) {
    for (int it = 0; it < iters && e == hipSuccess; ++it) e = hipGraphLaunch(exec, st);
    hipGraphExecDestroy(exec);
  }
  hipGraphDestroy(graph);
  return hip_code(e);
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

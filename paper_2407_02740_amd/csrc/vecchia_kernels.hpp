// Fused per-neighbourhood Vecchia kernel for gfx950 (CDNA4), FP64.
//
// One neighbourhood (observation i, its q = min(i, m) previously ordered
// nearest neighbours and itself, Section 2.1 Eq. 3) is processed by a group
// of 16 lanes: exactly one DPP row of a wave64, so every cross-lane step is
// a `row_newbcast` broadcast or a DPP butterfly inside the row.  A workgroup
// is one wave = 4 groups = 4 neighbourhoods in flight; the grid strides over
// the observation range.
//
// Matrix layout.  The neighbourhood covariance is K x K with K = 16*NS
// rounded down to the instantiated size (K >= m+1).  Local order: the q
// neighbours in rows 0..q-1, identity padding rows q..K-2 (exactly
// invariant: the padding block decouples from the rest), observation i last
// in row K-1 -- the row whose Cholesky entries give the conditional of y_i
// (Algorithm 1 reads index m).  Lane l of a group owns rows
//   slot s: row 16*s + l (s even) or 16*s + 15 - l (s odd),
// so slots pair up into rows of balanced length.  Each lane keeps its rows
// of the lower triangle in registers (A[], columns 0..min(16(s+1),K)-1).
//
// Steps per neighbourhood (Algorithm 1, with the "remaining operations" of
// the paper written out in the Cholesky-row form):
//   gather    locsub/ysub/Xsub of the next neighbourhood, prefetched into
//             registers during the current one; coordinates pre-scaled by
//             1/rho into LDS.
//   phase 1   covariance entries, one pair per lane per step with no idle
//             lanes: off-diagonal 16x16 blocks directly, and the two
//             triangular diagonal blocks of a slot pair folded into a
//             17-step loop (lane l takes row l's entry while u <= l, else
//             row 31-l's entry at column 32-u).  Each pair also leaves its
//             range-derivative factor sigma2 (-f'(h)/h) in LDS.
//   LDL^T     Sigma = Lt D Lt^T, right-looking in registers, column c's
//             pivot and entries broadcast with row_newbcast from their
//             owners; Lt is unit lower triangular, L = Lt D^(1/2).
//   solves    yt = Lt^-1 y, Xt = Lt^-1 X (forward, broadcasts); Lt to LDS
//             for the transposed access of ut = Lt^-T e_last (backward,
//             prefetched three steps ahead, interleaved with the forward
//             substitution).
//   phase 2   g_rho = (dSigma/drho) ut row by row: each lane sums over all
//             columns b of its rows a, the pair factors read from LDS
//             (static offsets, a zero slot on the diagonal), ut_b and z_b
//             uniform LDS reads one column ahead; nothing is scattered.
//   w         wt_rho = Lt^-1 g_rho, wt_tau2 = sigma2 Lt^-1 ut (dSigma/dtau2
//             = sigma2 I), w_sigma2 = e_last / sigma2 (dSigma/dsigma2 =
//             Sigma / sigma2); in the Cholesky-row form w_j = L^-1 dSigma_j u
//             with u = ut / sqrt(d_q), so w_j[l] = wt_j[l] / sqrt(d_l d_q).
//   sums      with Sy_j = sum_{l<q} w_j[l] Liy[l], SX_j likewise,
//             G_jk = sum_{l<q} w_j[l] w_k[l] (one DPP all-reduce), the self
//             row gives
//               logdet += log v,  ySy += Liy_q^2, XSX += LiX_q LiX_q^T,
//               ySX += Liy_q LiX_q,  dlogdet_j += w_j[q],
//               dySy_j += -2 Liy_q Sy_j - w_j[q] Liy_q^2,
//               dXSX_j += -(SX_j LiX_q^T + LiX_q SX_j^T) - w_j[q] LiX_q LiX_q^T,
//               dySX_j += -Sy_j LiX_q - Liy_q SX_j - w_j[q] Liy_q LiX_q,
//               ainfo_jk += G_jk + w_j[q] w_k[q] / 2,
//             (Liy_q = yt_q / sqrt(d_q), v = d_q) accumulated per group in
//             LDS by the self row's lane.
// The per-workgroup sums go to partials[block][nraw]; a second kernel adds
// them in a fixed order, so results are deterministic.  Other modes of the
// same kernel (adjoint, loglik only, kriging weights) and the batched
// work-queue schedule are described where they branch off below.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace vecchia {

#include "exp_table.inc"
#include "dpp_fmac.inc"

#ifdef VECCHIA_ISA_MARKS
#define VEC_MARK(x) asm volatile(";@@ " x)
#else
#define VEC_MARK(x)
#endif

// Profiling build only (-DVECCHIA_SECTION_TIMING): shader-clock cycles
// spent in each section of the per-neighbourhood loop, summed over waves.
#ifdef VECCHIA_SECTION_TIMING
constexpr int kSections = 12;
extern __device__ unsigned long long section_cycles[kSections];
#define VEC_TDECL                                  \
  __shared__ unsigned long long tsec_[kSections];  \
  if (threadIdx.x < kSections) tsec_[threadIdx.x] = 0; \
  unsigned long long tlast_ = clock64();           \
  int tcur_ = 0;
#define VEC_TMARK(idx)                                   \
  do {                                                   \
    __builtin_amdgcn_sched_barrier(0);                   \
    const unsigned long long tnow_ = clock64();          \
    if (threadIdx.x == 0) tsec_[tcur_] += tnow_ - tlast_; \
    tlast_ = tnow_;                                      \
    tcur_ = (idx);                                       \
  } while (0)
#define VEC_TFLUSH                                                      \
  do {                                                                  \
    VEC_TMARK(0);                                                       \
    __syncthreads();                                                    \
    if (threadIdx.x < kSections) atomicAdd(&section_cycles[threadIdx.x], tsec_[threadIdx.x]); \
  } while (0)
#else
#define VEC_TDECL
#define VEC_TMARK(idx)
#define VEC_TFLUSH
#endif

constexpr int kGroupsPerBlock = 4;
constexpr int kThreads = 64;

// nu codes: 0 -> 1/2, 1 -> 3/2, 2 -> 5/2
constexpr int nraw_of(int p, int P) { return 2 + p * p + p + P * (2 + p * p + p) + P * P; }

// What one pass of the fused kernel accumulates per neighbourhood.
//   kModeSums     the loglik, gradient and Fisher-information sums
//                 (nraw_of(p, P) doubles, layout of vec_raw_sums).
//   kModeAdjoint  the gradient at a given beta by the reverse-mode
//                 expression (logdet, r'S r, grad[P]; r = y - X beta).
//   kModeLoglik   the sums of Algorithm 1 alone (logdet, ySy, XSX, ySX).
//   kModeWeights  the sums of kModeLoglik, and per observation its kriging
//                 weights b (in NNarray column order) and log(v / sigma2),
//                 the conditional variance in correlation units.
constexpr int kModeSums = 0, kModeAdjoint = 1, kModeLoglik = 2, kModeWeights = 3;
constexpr int nraw_mode(int mode, int p, int P) {
  return mode == kModeSums ? nraw_of(p, P) : (mode == kModeAdjoint ? 2 + P : nraw_of(p, 0));
}

template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}

// Value of x held by lane LANE of this lane's 16-lane DPP row.
template <int LANE>
__device__ __forceinline__ double bcast(double x) {
  return __builtin_amdgcn_mov_dpp(x, 0x150 + LANE, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
  return __builtin_amdgcn_mov_dpp(x, CTRL, 0xF, 0xF, false);
}

// Sum over the 16 lanes of the DPP row, identical bits on every lane:
// xor-1, xor-2 (quad_perm), 8-lane half mirror, 16-lane mirror.
__device__ __forceinline__ double row_allreduce(double x) {
  x += dpp<0xB1>(x);
  x += dpp<0x4E>(x);
  x += dpp<0x141>(x);
  x += dpp<0x140>(x);
  return x;
}

// 1/sqrt(x) for x > 0: hardware estimate refined by one Newton step with the
// second-order term, y1 = y0 (1 + e/2 + 3e^2/8), e = 1 - x y0^2.
__device__ __forceinline__ double rsqrt_refined(double x) {
  const double y0 = __builtin_amdgcn_rsq(x);
  const double e = __builtin_fma(-(x * y0), y0, 1.0);
  return __builtin_fma(y0 * e, __builtin_fma(0.375, e, 0.5), y0);
}

// 1/x for x > 0: hardware estimate refined to y0 (1 + e + e^2), e = 1 - x y0.
__device__ __forceinline__ double rcp_refined(double x) {
  const double y0 = __builtin_amdgcn_rcp(x);
  const double e = __builtin_fma(-x, y0, 1.0);
  return __builtin_fma(y0, __builtin_fma(e, e, e), y0);
}

template <int K>
struct Geo {
  static constexpr int NS = (K + 15) / 16;
  static constexpr int KP = 16 * NS;
  static constexpr int len(int s) { return (16 * (s + 1) < K) ? 16 * (s + 1) : K; }
  static constexpr int off(int s) {
    int o = 0;
    for (int t = 0; t < s; ++t) o += len(t);
    return o;
  }
  static constexpr int NL = off(NS);
  static constexpr int slot_of(int r) { return r / 16; }
  // Factorisation column c updates rows c+1..K-1 in groups of up to four
  // rows that lie in one 16-row block: first row of group g, group count.
  static constexpr int gstart(int c, int g) {
    int r = c + 1;
    for (int t = 0; t < g && r < K; ++t) {
      const int bend = (16 * (r / 16 + 1) < K) ? 16 * (r / 16 + 1) : K;
      r += (bend - r < 4) ? bend - r : 4;
    }
    return r;
  }
  static constexpr int ngroups(int c) {
    int g = 0;
    while (gstart(c, g) < K) ++g;
    return g;
  }
  static constexpr int lane_of(int r) {
    return ((r / 16) & 1) ? 16 * (r / 16) + 15 - r : r - 16 * (r / 16);
  }
};

// LDS ordering between the lanes of one wavefront.  A workgroup is a single
// wave64 and LDS instructions of a wave complete in issue order, so a
// wavefront-scope fence (compiler ordering, no wait) is all that cross-lane
// communication through LDS needs.
__device__ __forceinline__ void wave_lds_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

__device__ __forceinline__ int row_of(int s, int l) { return 16 * s + ((s & 1) ? 15 - l : l); }

// Squared distances are accumulated from kH2Floor instead of 0, so that
// coincident locations give h ~ 1e-150 and a finite 1/h (every use
// multiplies 1/h by a squared coordinate difference that is then 0); for any
// h2 above 1e-284 the floor does not change the sum.
constexpr double kH2Floor = 1e-300;

// h = sqrt(h2) and 1/h for h2 >= kH2Floor.
__device__ __forceinline__ void dist_from_sq(double h2, double& h, double& hinv) {
  const double r = rsqrt_refined(h2);
  h = h2 * r;
  hinv = r;
}

struct CovCoef {
  double sigma2, diag;  // sigma2, sigma2 * (1 + tau2)
  double c1, c2;        // f = (1 + c1 h + c2 h^2) e^-h
  double a0, a1, a2;    // -f'(h)/h = (a0 + a1 h + a2/h) e^-h
  double ir[2];         // 1/range per group
  // gather: scaled coordinate k of a row is locs[row][col[k]] * sc[k]
  // (isotropic: coordinate k, zero beyond d; space-time: spatial
  // coordinates 0..d-2 in z[0..d-2], time coordinate d-1 in z[3])
  int col[4];
  double sc[4];
};

// Batched launches.  The device plan holds, per dataset, kSetFields int64:
// offset of its rows in locs / y / X, offset of its NNarray block, n, m,
// smoothness code, size class, first partial row and number of tiles; and
// per size class the datasets of the class in queue order with the prefix
// sum of their tiles.  Every tile is a contiguous range of one dataset's
// observations and owns one row of partial sums, so per-dataset results do
// not depend on which workgroup took which tile.
constexpr int kSetFields = 8;
enum SetField { kSetObs = 0, kSetNN, kSetN, kSetM, kSetNu, kSetClass, kSetRow, kSetTiles };

struct BatchClass {
  const int64_t* sets;          // [nsets][kSetFields]
  const int32_t* class_sets;    // datasets of this class, in queue order
  const int64_t* class_prefix;  // [count + 1]: first tile of each dataset, total last
  unsigned int* counter;        // work-queue head, zero before the launch
  int64_t row0;                 // partial row of the class's first tile
  int32_t count;                // datasets in the class
  int32_t tile;                 // neighbourhoods per tile
};

struct SumsArgs {
  int m, d, nspace, nu;
  const double* locs;
  const int32_t* NN;
  const double* y;
  const double* X;
  const double* covparms;  // [P]; batched: [nsets][P]
  const double* beta;      // adjoint mode: [p]
  int64_t i0, i1;          // observation range (single problem)
  double* partials;        // [rows][nraw]
  int32_t* status;         // [2]; batched: [nsets][2]
  double* rows_out;        // weights mode: [i1 - i0][m + 1]
  const int32_t* index;    // optional: observations at positions [i0, i1) of this list
  int64_t n;               // observations of the problem (bounds of index entries)
  int64_t nn_row0;         // observation whose NNarray row is NN[0] (0: the whole array)
  // short_rows != 0: a -1 among the first min(i, m) neighbour columns is a
  // missing neighbour (a padding row), and a row whose column 0 is -1 is
  // skipped (it contributes nothing and is not an error)
  int32_t short_rows;
  BatchClass batch;
};

// BATCH = false: one problem, the grid strides over observations [i0, i1)
// and each workgroup writes one partial row.  BATCH = true: a persistent
// grid takes tiles from the class's work queue until it is empty.
template <int K, int PC, int NG, int MODE, bool BATCH>
__global__ __launch_bounds__(kThreads) void sums_kernel(const SumsArgs a) {
  using G = Geo<K>;
  constexpr int NS = G::NS;
  constexpr int KP = G::KP;
  constexpr int NL = G::NL;
  constexpr int P = NG + 2;   // sigma2, ranges, tau2
  constexpr int NR = NG + 1;  // parameters whose w has entries above the self row
  constexpr bool kFull = MODE == kModeSums;
  constexpr bool kAdj = MODE == kModeAdjoint;
  constexpr bool kLik = MODE == kModeLoglik;
  constexpr bool kWts = MODE == kModeWeights;
  constexpr bool kDeriv = kFull || kAdj;  // derivative work: pair factors and phase 2
  // Above K = 41 the stored pair factors would take the LDS of two more
  // workgroups per CU: phase 2 recomputes them from the coordinates instead.
  constexpr bool kRecomp = kDeriv && K > 41;
  constexpr bool kStoreF = kDeriv && !kRecomp;
  constexpr int NRAW = nraw_mode(MODE, PC, P);
  constexpr int RC = kAdj ? 1 : 1 + PC;  // right-hand sides of the forward substitution
  constexpr int LPN = K * (K - 1) / 2;  // strictly lower L, index r(r-1)/2 + c
  static_assert(K % 16 != 0, "rows >= K serve as spare rows");
  constexpr int SS = G::slot_of(K - 1);
  constexpr int LS = G::lane_of(K - 1);
  constexpr int NGR = NR * (NR + 1) / 2;
  constexpr int NPART = NR + NR * PC + NGR;

  // per-row record: scaled coordinates z[0..3] (space-time: time in z[3]),
  // u, and the row's inverse pivot 1/d_r (0 for rows >= K).  Rows that are
  // never read as a partner -- the spare rows of an unpaired last slot --
  // share one sink row at RROWS.
  constexpr int RZ = 0, RU = 4, RI = 5;
  constexpr int RS = 6;  // row stride, 16-byte aligned
  constexpr int RROWS = (K > 16 * (NS - (NS & 1))) ? K : 16 * (NS - (NS & 1));
  constexpr int RREC = RROWS + (NS & 1);  // + the sink row (odd NS only)
  __shared__ double rec[kGroupsPerBlock][RREC][RS];
  // rows 0..K-1 packed at r(r-1)/2 (stores of a row run past its diagonal
  // into later rows, see the store below), then a sink for rows >= K
  constexpr int LPS = LPN + 1 + K;
  // Above K = 21 the back substitutions run row by row on the factor in
  // registers, one 16-lane sum per row, instead of on a copy of Lt in LDS
  // (measured as fast at K = 31, and its LDS holds the pair factors).
  constexpr bool kRowBack = K > 21;
  __shared__ double Lp[kGroupsPerBlock][(kLik || kRowBack) ? 1 : LPS];
  __shared__ double acc[kGroupsPerBlock][NRAW];
  // running product of conditional variances (mantissa, exponent)
  __shared__ double vprod[kGroupsPerBlock][2];
  // per pair (r, c), c <= r < K, at r(r+1)/2 + c: sigma2 (-f'(h)/h), from
  // which every range derivative of the pair follows (on the diagonal the
  // squared coordinate differences that multiply it are 0); then a sink of
  // KP entries for the rows >= K and for the upper-triangle steps of an
  // unpaired last slot
  constexpr int NQ = K * (K + 1) / 2;
  // Space-time up to K = 31: two finished factors per pair instead,
  // sigma2 (-f'(h)/h) times the squared spatial and time differences (the
  // range derivatives up to 1/rho), interleaved at 2 (r(r+1)/2 + c); the
  // sink is the single pair at NQ, every index clamped to it where it could
  // pass it.  (At K = 31 with three covariates the larger sums would take
  // the workgroup past a quarter of the CU's LDS: one factor there.)
  constexpr bool kTwoF = kStoreF && NG == 2 && (K <= 21 || (K <= 31 && PC <= 2));
  __shared__ double sfv[kGroupsPerBlock][kStoreF ? (kTwoF ? 2 * (NQ + 1) : NQ + KP) : 2];

  const int lane = threadIdx.x & 15;
  const int grp = threadIdx.x >> 4;
  constexpr double kFar = 1e30;
  // Lp offsets of this lane's rows: where its row r starts (the sink for
  // rows >= K, and for row 0, which has no entries and would share its start
  // with row 1), and its column r in the rows below
  int lrow_base[NS], lcol_base[NS];
  // and the start of its pair factors (the sink for rows >= K), and its row
  // record (the sink row for rows >= RROWS)
  int qrow_base[NS], rrow[NS];
  sfor<0, NS>([&](auto s_) {
    const int r = row_of(s_.value, lane);
    lrow_base[s_.value] = (r >= 1 && r < K) ? r * (r - 1) / 2 : LPN + 1;
    lcol_base[s_.value] = r;
    qrow_base[s_.value] = (r < K) ? r * (r + 1) / 2 : NQ;
    rrow[s_.value] = (r < RROWS) ? r : RROWS;
  });

  // the problem of the current tile (BATCH: one dataset's slice)
  const int d = a.d;
  int m = a.m, nu = a.nu;
  const double* __restrict__ locs = a.locs;
  const int32_t* __restrict__ NN = a.NN;
  const double* __restrict__ y = a.y;
  const double* __restrict__ X = a.X;
  const double* __restrict__ covparms = a.covparms;
  int32_t* __restrict__ status = a.status;
  int64_t i0 = a.i0, total = a.i1 - a.i0;

  __shared__ double exptab[64];
  CovCoef cf;
  double inv_sigma2;
  double bt[PC];
  auto set_params = [&]() {
    cf.sigma2 = covparms[0];
    const double tau2 = covparms[P - 1];
    cf.diag = cf.sigma2 * (1.0 + tau2);
    cf.ir[0] = 1.0 / covparms[1];
    cf.ir[1] = (NG == 2) ? 1.0 / covparms[2] : cf.ir[0];
    cf.c1 = (nu >= 1) ? 1.0 : 0.0;
    cf.c2 = (nu == 2) ? 1.0 / 3.0 : 0.0;
    cf.a0 = (nu == 0) ? 0.0 : ((nu == 1) ? 1.0 : 1.0 / 3.0);
    cf.a1 = (nu == 2) ? 1.0 / 3.0 : 0.0;
    cf.a2 = (nu == 0) ? 1.0 : 0.0;
    inv_sigma2 = 1.0 / cf.sigma2;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (NG == 2 && k == 3) {
        cf.col[k] = d - 1;
        cf.sc[k] = cf.ir[1];
      } else {
        const int dl = (NG == 2) ? d - 1 : d;  // coordinates scaled by the first range
        cf.col[k] = (k < dl) ? k : dl - 1;
        cf.sc[k] = (k < dl) ? cf.ir[0] : 0.0;
      }
    }
#pragma unroll
    for (int t = 0; t < PC; ++t) bt[t] = kAdj ? a.beta[t] : 0.0;
    // 2^(j/64) scaled by sigma2: every covariance entry carries the factor
    exptab[threadIdx.x] = kExp2Tab[threadIdx.x] * cf.sigma2;
    wave_lds_fence();
  };

  for (int e = threadIdx.x; e < kGroupsPerBlock * NRAW; e += kThreads) (&acc[0][0])[e] = 0.0;
  for (int e = threadIdx.x; e < kGroupsPerBlock * RREC; e += kThreads)
    rec[e / RREC][e % RREC][RI] = 0.0;
  static_assert(kThreads == 64, "one table entry per thread");
  __syncthreads();
  if (threadIdx.x < kGroupsPerBlock) {
    vprod[threadIdx.x][0] = 1.0;
    vprod[threadIdx.x][1] = 0.0;
  }

  VEC_TDECL
  const int64_t stride = BATCH ? kGroupsPerBlock : (int64_t)gridDim.x * kGroupsPerBlock;
  const int64_t first = BATCH ? 0 : (int64_t)blockIdx.x * kGroupsPerBlock;

  // Neighbour indices of observation ii for this lane's rows: id = -1 for
  // padding rows (and rows >= K), ii for the self row.  Only valid columns
  // 1..q of the NNarray row are read (column 0 otherwise).  Neighbours are
  // earlier observations; rows appended after the observed ones (nn_row0 >
  // 0, prediction points) may only name observed points j < nn_row0.
  auto fetch_ids = [&](int64_t ii, int lan, int64_t(&id)[NS], bool& bad, bool& skip) {
    const int32_t* row = NN + (ii - a.nn_row0) * (int64_t)(m + 1);
    const int32_t head = row[0];
    skip = a.short_rows && head == -1;
    const int qq = skip ? 0 : (int)(ii < (int64_t)m ? ii : (int64_t)m);
    const int64_t jend = (a.nn_row0 > 0) ? a.nn_row0 : ii;
    bad = !skip && (head != (int32_t)ii);
    sfor<0, NS>([&](auto s_) {
      constexpr int s = s_.value;
      const int r = row_of(s, lan);
      const bool nb = r < qq;
      const int64_t j = row[nb ? 1 + r : 0];
      const bool okj = (j >= 0) && (j < jend);
      bad = bad || (nb && !okj && !(a.short_rows && j == -1));
      id[s] = (r == K - 1) ? ii : ((nb && okj) ? j : (int64_t)-1);
    });
  };
  // Raw coordinates, y and X of those rows (row ii stands in for padding).
  auto fetch_vals = [&](int64_t ii, const int64_t(&id)[NS], double(&zv)[NS][4],
                        double(&yv)[NS], double(&xv)[NS][PC]) {
    sfor<0, NS>([&](auto s_) {
      constexpr int s = s_.value;
      const int64_t ids = (id[s] >= 0) ? id[s] : ii;
#pragma unroll
      for (int k = 0; k < 4; ++k) zv[s][k] = locs[ids * d + cf.col[k]];
      yv[s] = y[ids];
#pragma unroll
      for (int t = 0; t < PC; ++t) xv[s][t] = X[ids * PC + t];
    });
  };
  // observation of this group at position bse of the range; with an index
  // list the positions index it (entries outside [0, n) read observation 0
  // and are reported as a malformed row by index_bad)
  auto obs_of = [&](int64_t bse) -> int64_t {
    const int64_t pos = i0 + ((bse + grp < total) ? bse + grp : total - 1);
    if (a.index == nullptr) return pos;
    const int64_t v = a.index[pos];
    return (v >= 0 && v < a.n) ? v : 0;
  };
  auto index_bad = [&](int64_t bse) -> bool {
    if (a.index == nullptr) return false;
    const int64_t v = a.index[i0 + ((bse + grp < total) ? bse + grp : total - 1)];
    return !(v >= 0 && v < a.n);
  };

  // Software pipeline over the wave's neighbourhoods: the next NNarray row
  // is loaded at the top of an iteration and the next coordinates, y and X
  // after phase 1, so each gather finds its inputs in registers.
  int64_t idc[NS];
  bool badc = false, skipc = false;
  double zv[NS][4], yv[NS], xv[NS][PC];

  // sums of the groups (logdet from the running product) into one row of
  // partials, then the accumulators start again
  auto flush = [&](double* __restrict__ dst) {
    __syncthreads();
    if (threadIdx.x < kGroupsPerBlock) {
      acc[threadIdx.x][0] = log(vprod[threadIdx.x][0]) + vprod[threadIdx.x][1] * 0.6931471805599453;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < NRAW; e += kThreads)
      dst[e] = ((acc[0][e] + acc[1][e]) + acc[2][e]) + acc[3][e];
    if constexpr (BATCH) {
      __syncthreads();
      for (int e = threadIdx.x; e < kGroupsPerBlock * NRAW; e += kThreads) (&acc[0][0])[e] = 0.0;
      if (threadIdx.x < kGroupsPerBlock) {
        vprod[threadIdx.x][0] = 1.0;
        vprod[threadIdx.x][1] = 0.0;
      }
      __syncthreads();
    }
  };
  // next tile of the class's work queue (wave-uniform)
  auto grab = [&]() -> int64_t {
    unsigned int t = 0;
    if (threadIdx.x == 0) t = atomicAdd(a.batch.counter, 1u);
    return (int64_t)__builtin_amdgcn_readfirstlane((int)t);
  };

  int64_t tile = BATCH ? grab() : 0;
  for (;;) {
  if constexpr (BATCH) {
    const BatchClass& bc = a.batch;
    if (tile >= bc.class_prefix[bc.count]) break;
    // the dataset of the tile: last k with class_prefix[k] <= tile
    int lo = 0, hi = bc.count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (bc.class_prefix[mid] <= tile) lo = mid; else hi = mid - 1;
    }
    const int ds = bc.class_sets[lo];
    const int64_t* sd = bc.sets + (int64_t)ds * kSetFields;
    const int64_t lt = tile - bc.class_prefix[lo];
    locs = a.locs + sd[kSetObs] * d;
    y = a.y + sd[kSetObs];
    X = a.X + sd[kSetObs] * PC;
    NN = a.NN + sd[kSetNN];
    m = (int)sd[kSetM];
    nu = (int)sd[kSetNu];
    i0 = lt * bc.tile;
    total = (sd[kSetN] - i0 < bc.tile) ? sd[kSetN] - i0 : bc.tile;
    covparms = a.covparms + (int64_t)ds * P;
    status = a.status + 2 * ds;
  }
  set_params();
  if (first < total) {
    const int64_t ii = obs_of(first);
    fetch_ids(ii, lane, idc, badc, skipc);
    fetch_vals(ii, idc, zv, yv, xv);
  }

  for (int64_t base = first; base < total; base += stride) {
    // an opaque copy of the lane id per iteration keeps the many
    // lane-dependent predicates from being hoisted out of the loop
    int l = lane;
    asm volatile("" : "+v"(l));
    const bool active = base + grp < total && !skipc;
    const int64_t i = obs_of(base);
    const bool badidx = index_bad(base);
    const int q = (int)(i < (int64_t)m ? i : (int64_t)m);
    const bool more = base + stride < total;
    const int64_t inext = more ? obs_of(base + stride) : i;
    int64_t idn[NS];
    sfor<0, NS>([&](auto s_) { idn[s_.value] = -1; });
    bool badn = false, skipn = false;
    bool badnn = badc;
    bool badval = false;

    VEC_MARK("gather");
    VEC_TMARK(1);
    // ---------------- gather ----------------
    // Rows without an observation (padding q <= r < K-1, rows >= K) get
    // coordinates kFar*(1+r) apart from everything: their covariance with
    // any other row is exp(-h) = 0 exactly, so the padding block decouples
    // with no masking anywhere below.
    double zo[NS][4];
    double rhs[RC][NS];
    sfor<0, NS>([&](auto s_) {
      constexpr int s = s_.value;
      const int r = row_of(s, l);
      const bool has = idc[s] >= 0;
      // scaled coordinates (the column map of set_params); a non-finite
      // coordinate makes the sum non-finite
      double zc[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) zc[k] = zv[s][k] * cf.sc[k];
      badval |= has && !__builtin_isfinite((zc[0] + zc[1]) + (zc[2] + zc[3]));
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        zo[s][k] = has ? zc[k] : ((k == 0) ? kFar * (double)(1 + r) : 0.0);
        rec[grp][rrow[s]][RZ + k] = zo[s][k];
      }
      if constexpr (kAdj) {
        // residual at the given beta
        double rv = yv[s];
#pragma unroll
        for (int t = 0; t < PC; ++t) rv = __builtin_fma(-xv[s][t], bt[t], rv);
        rhs[0][s] = has ? rv : 0.0;
      } else {
        rhs[0][s] = has ? yv[s] : 0.0;
#pragma unroll
        for (int t = 0; t < PC; ++t) rhs[1 + t][s] = has ? xv[s][t] : 0.0;
      }
    });
    // next NNarray row, in flight during phase 1
    if (more) fetch_ids(inext, l, idn, badn, skipn);
    wave_lds_fence();

    // Covariance of two pairs of scaled locations (evaluated side by side so
    // that their latencies overlap), and each pair's range-derivative factor
    // sigma2 (-f'(h)/h) stored at sfv[idx].  exp(-h) is table driven: with
    // -h = (64 m + j) ln2/64 + r, |r| <= ln2/128,
    //   sigma2 e^-h = 2^m * T[j] * (1 + q),  T[j] = sigma2 2^(j/64),
    //   q = r + r^2/2 + ... + r^5/120 (truncation below 4e-17 relative),
    // formed as T + T q; -h is clamped at -800 so that 2^m underflows to 0.
    // kExpo (smoothness 1/2): f = e^-h and -f'(h)/h = e^-h / h, the general
    // forms with c1 = c2 = a0 = a1 = 0 and a2 = 1 written without their
    // zero terms (the same values bit for bit).
    auto pair_eval2 = [&](auto expo_, const double* za0, const double* zb0, int idx0,
                          const double* za1, const double* zb1, int idx1, double& v0,
                          double& v1) {
      constexpr bool kExpo = decltype(expo_)::value;
      double h20 = kH2Floor, h21 = kH2Floor;
      double hs0 = 0.0, hs1 = 0.0, ht0 = 0.0, ht1 = 0.0;  // kTwoF: space and time parts
      if constexpr (kTwoF) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double t0 = za0[k] - zb0[k];
          const double t1 = za1[k] - zb1[k];
          hs0 = __builtin_fma(t0, t0, hs0);
          hs1 = __builtin_fma(t1, t1, hs1);
        }
        const double u0 = za0[3] - zb0[3], u1 = za1[3] - zb1[3];
        ht0 = u0 * u0;
        ht1 = u1 * u1;
        h20 = (hs0 + kH2Floor) + ht0;
        h21 = (hs1 + kH2Floor) + ht1;
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double t0 = za0[k] - zb0[k];
          const double t1 = za1[k] - zb1[k];
          h20 = __builtin_fma(t0, t0, h20);
          h21 = __builtin_fma(t1, t1, h21);
        }
      }
      double hh0, hi0, hh1, hi1;
      dist_from_sq(h20, hh0, hi0);
      dist_from_sq(h21, hh1, hi1);
      const double x0 = fmax(-hh0, -800.0), x1 = fmax(-hh1, -800.0);
      const double n0 = rint(x0 * kInvLn2x64), n1 = rint(x1 * kInvLn2x64);
      const int i0n = (int)n0, i1n = (int)n1;
      const double T0 = exptab[i0n & 63], T1 = exptab[i1n & 63];
      double r0 = __builtin_fma(-n0, kLn2d64Hi, x0), r1 = __builtin_fma(-n1, kLn2d64Hi, x1);
      r0 = __builtin_fma(-n0, kLn2d64Lo, r0);
      r1 = __builtin_fma(-n1, kLn2d64Lo, r1);
      double q0 = __builtin_fma(r0, 1.0 / 120.0, 1.0 / 24.0), q1 = __builtin_fma(r1, 1.0 / 120.0, 1.0 / 24.0);
      q0 = __builtin_fma(q0, r0, 1.0 / 6.0);
      q1 = __builtin_fma(q1, r1, 1.0 / 6.0);
      q0 = __builtin_fma(q0, r0, 0.5);
      q1 = __builtin_fma(q1, r1, 0.5);
      q0 = __builtin_fma(q0, r0, 1.0);
      q1 = __builtin_fma(q1, r1, 1.0);
      q0 *= r0;
      q1 *= r1;
      const double sE0 = ldexp(__builtin_fma(T0, q0, T0), i0n >> 6);
      const double sE1 = ldexp(__builtin_fma(T1, q1, T1), i1n >> 6);
      const double sF0 = kExpo ? sE0 * hi0
                               : sE0 * __builtin_fma(cf.a1, hh0, __builtin_fma(cf.a2, hi0, cf.a0));
      const double sF1 = kExpo ? sE1 * hi1
                               : sE1 * __builtin_fma(cf.a1, hh1, __builtin_fma(cf.a2, hi1, cf.a0));
      if constexpr (kTwoF) {
        const int j0 = idx0 < NQ ? idx0 : NQ, j1 = idx1 < NQ ? idx1 : NQ;
        sfv[grp][2 * j0] = sF0 * hs0;
        sfv[grp][2 * j0 + 1] = sF0 * ht0;
        sfv[grp][2 * j1] = sF1 * hs1;
        sfv[grp][2 * j1 + 1] = sF1 * ht1;
      } else if constexpr (kStoreF) {
        // isotropic: the finished dSigma/drho entry, sF h^2 / rho (h^2 without
        // the floor, so that it is exactly 0 on the diagonal and at
        // coincident locations)
        sfv[grp][idx0] = (NG == 1) ? sF0 * (h20 - kH2Floor) * cf.ir[0] : sF0;
        sfv[grp][idx1] = (NG == 1) ? sF1 * (h21 - kH2Floor) * cf.ir[0] : sF1;
      }
      v0 = kExpo ? sE0 : sE0 * __builtin_fma(hh0, __builtin_fma(hh0, cf.c2, cf.c1), 1.0);
      v1 = kExpo ? sE1 : sE1 * __builtin_fma(hh1, __builtin_fma(hh1, cf.c2, cf.c1), 1.0);
    };
    auto pidx = [](int r, int c) { return r * (r + 1) / 2 + c; };

    VEC_MARK("phase1");
    VEC_TMARK(2);
    // ---------------- phase 1: covariance ----------------
    // Entries above the diagonal of a lane's rows are never read, so every
    // step may write its value into both candidate registers.
    double A[NL];
    sfor<0, NL>([&](auto e_) { A[e_.value] = 0.0; });
    // one copy of the phase for smoothness 1/2 and one for the others
    auto phase1 = [&](auto expo_) {
    // off-diagonal 16x16 blocks: slot s rows x columns of block t < s, two
    // columns per step, partner coordinates read one step ahead
    sfor<1, NS>([&](auto s_) {
      constexpr int s = s_.value;
      sfor<0, s>([&](auto t_) {
        constexpr int t = t_.value;
        double zn[2][4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          zn[0][k] = rec[grp][16 * t][RZ + k];
          zn[1][k] = rec[grp][16 * t + 1][RZ + k];
        }
        sfor<0, 8>([&](auto cc_) {
          constexpr int c = 16 * t + 2 * cc_.value;
          double zc[2][4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            zc[0][k] = zn[0][k];
            zc[1][k] = zn[1][k];
          }
          if constexpr (cc_.value + 1 < 8) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              zn[0][k] = rec[grp][c + 2][RZ + k];
              zn[1][k] = rec[grp][c + 3][RZ + k];
            }
          }
          const int r = row_of(s, l);
          pair_eval2(expo_, zo[s], zc[0], qrow_base[s] + c, zo[s], zc[1], qrow_base[s] + c + 1, A[G::off(s) + c],
                     A[G::off(s) + c + 1]);
        });
      });
    });
    // diagonal blocks of slots (2t, 2t+1) folded into 17 steps (two per
    // evaluation): lane l takes row 16 s0 + l's entry at column 16 s0 + u
    // while u <= l, else row 16 s1 + 15 - l's entry at column 16 s1 + 16 - u
    sfor<0, NS / 2>([&](auto t_) {
      constexpr int s0 = 2 * t_.value;
      constexpr int s1 = s0 + 1;
      const int ra = 16 * s0 + l, rb = 16 * s1 + 15 - l;
      const int qa = (ra < K) ? ra * (ra + 1) / 2 : NQ, qb = (rb < K) ? rb * (rb + 1) / 2 : NQ;
      auto locate = [&](auto u_, int& r, int& c, int& q, double(&zr)[4], double(&zc)[4]) {
        constexpr int u = decltype(u_)::value;
        const bool first = (u <= l);
        c = first ? 16 * s0 + u : 16 * s1 + 16 - u;
        r = first ? ra : rb;
        q = first ? qa + (16 * s0 + u) : qb + (16 * s1 + 16 - u);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          zr[k] = rec[grp][r][RZ + k];
          zc[k] = rec[grp][c][RZ + k];
        }
      };
      auto store = [&](auto u_, int r, int c, double off) {
        constexpr int u = decltype(u_)::value;
        const double v = (c == r) ? cf.diag : off;
        if constexpr (u <= 15) A[G::off(s0) + 16 * s0 + u] = v;
        if constexpr (u >= 1 && 16 * s1 + 16 - u < K) A[G::off(s1) + 16 * s1 + 16 - u] = v;
      };
      int rn[2], cn[2], qn[2];
      double zrn[2][4], zcn[2][4];
      locate(std::integral_constant<int, 0>{}, rn[0], cn[0], qn[0], zrn[0], zcn[0]);
      locate(std::integral_constant<int, 1>{}, rn[1], cn[1], qn[1], zrn[1], zcn[1]);
      sfor<0, 9>([&](auto w_) {
        constexpr int u = 2 * w_.value;          // steps u and u + 1 (17 steps)
        int r[2] = {rn[0], rn[1]}, c[2] = {cn[0], cn[1]}, q[2] = {qn[0], qn[1]};
        double zr[2][4], zc[2][4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          zr[0][k] = zrn[0][k];
          zc[0][k] = zcn[0][k];
          zr[1][k] = zrn[1][k];
          zc[1][k] = zcn[1][k];
        }
        if constexpr (u + 2 < 17) locate(std::integral_constant<int, u + 2>{}, rn[0], cn[0], qn[0], zrn[0], zcn[0]);
        if constexpr (u + 3 < 17) locate(std::integral_constant<int, u + 3>{}, rn[1], cn[1], qn[1], zrn[1], zcn[1]);
        double off0, off1;
        if constexpr (u + 1 < 17) {
          pair_eval2(expo_, zr[0], zc[0], q[0], zr[1], zc[1], q[1], off0, off1);
          store(std::integral_constant<int, u>{}, r[0], c[0], off0);
          store(std::integral_constant<int, u + 1>{}, r[1], c[1], off1);
        } else {
          // last (odd) step: the second slot of the evaluation repeats it
          pair_eval2(expo_, zr[0], zc[0], q[0], zr[0], zc[0], q[0], off0, off1);
          store(std::integral_constant<int, u>{}, r[0], c[0], off0);
        }
      });
    });
    // unpaired last slot (odd NS): its triangle directly
    if constexpr (NS & 1) {
      constexpr int s = NS - 1;
      sfor<0, G::len(s) - 16 * s>([&](auto u_) {
        constexpr int c = 16 * s + u_.value;
        const int r = row_of(s, l);
        double zc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) zc[k] = rec[grp][c][RZ + k];
        double off, dup;
        // steps past the lane's row (upper triangle) write the sink
        pair_eval2(expo_, zo[s], zc, (c <= r) ? qrow_base[s] + c : NQ + c, zo[s], zc, NQ, off,
                   dup);
        A[G::off(s) + c] = (c == r) ? cf.diag : off;
      });
    }
    };
    // (the 61-row kernels, at the register limit already, keep one copy)
    if (K <= 41 && nu == 0)
      phase1(std::true_type{});
    else
      phase1(std::false_type{});

    VEC_MARK("cholesky");
    VEC_TMARK(3);
    // ---------------- LDL^T factorisation (right-looking, in registers) ----------------
    // Sigma = Lt D Lt^T with Lt unit lower triangular, so L = Lt D^(1/2) and
    // every substitution below runs on Lt without divisions.  Column c:
    // broadcast the pivot d_c and each unscaled entry A[r][c]; rows update
    // with Lt[row][c] = A[row][c] / d_c.  The owner of row r keeps 1/d_r.
    double idg[NS];
    bool notpd = false;
    double vself = 1.0;
    // One group of column c's updates: rows r0 .. r0+n-1 of block b, then
    // the next group.  After the first group the next column's pivot is
    // broadcast and its reciprocal started, so that chain runs under the
    // remaining updates.
    auto chol_group = [&](auto c_, auto r0_, auto nL_, double& dvn, double& rin) {
      constexpr int c = decltype(c_)::value, r0 = decltype(r0_)::value;
      constexpr int b = r0 / 16;
      constexpr int bend = (16 * (b + 1) < K) ? 16 * (b + 1) : K;
      constexpr int n = (bend - r0 < 4) ? bend - r0 : 4;
      constexpr int NSL = NS - b;
      double acc[n][NSL], src[n], mul[NSL];
      sfor<0, n>([&](auto i_) {
        src[i_.value] = A[G::off(b) + c];
        sfor<0, NSL>([&](auto j_) { acc[i_.value][j_.value] = A[G::off(b + j_.value) + r0 + i_.value]; });
      });
      sfor<0, NSL>([&](auto j_) { mul[j_.value] = nL_[b + j_.value]; });
      dpp_fmac<n, NSL, G::lane_of(r0), G::lane_of(r0 + (n > 1 ? 1 : 0)),
               G::lane_of(r0 + (n > 2 ? 2 : 0)), G::lane_of(r0 + (n > 3 ? 3 : 0))>(acc, src, mul);
      sfor<0, n>([&](auto i_) {
        sfor<0, NSL>([&](auto j_) { A[G::off(b + j_.value) + r0 + i_.value] = acc[i_.value][j_.value]; });
      });
      if constexpr (r0 == c + 1) {
        dvn = dpp_bcast<G::lane_of(c + 1)>(A[G::off((c + 1) / 16) + c + 1]);
        rin = rcp_refined(dvn);
      }
    };
    // pivot of the next column: taken (and its reciprocal started) right
    // after the first update group of the current one, so that chain runs
    // under the remaining updates
    double dv_next = dpp_bcast<G::lane_of(0)>(A[G::off(0) + 0]);
    double ri_next = rcp_refined(dv_next);
    sfor<0, K>([&](auto c_) {
      constexpr int c = c_.value;
      constexpr int sc = c / 16;
      const double dv = dv_next;
      notpd |= !(dv > 0.0);
      const double ri = ri_next;
      if constexpr (c == K - 1) vself = dv;
      rec[grp][c][RI] = ri;  // the same value from every lane
      // -Lt[row][c] = -A[row][c] / d_c for this lane's rows
      double nL[NS];
      sfor<0, NS>([&](auto s_) {
        constexpr int s = s_.value;
        if constexpr (16 * s + 15 > c) nL[s] = A[G::off(s) + c] * (-ri);
      });
      // rows r = c+1.. in groups of up to four rows of one 16-row block:
      // A[row][r] += (A[r][c] broadcast from its owner) * (-Lt[row][c]) for
      // the slots from that block on, the broadcast folded into the
      // multiply-add
      sfor<0, G::ngroups(c)>([&](auto g_) {
        chol_group(c_, std::integral_constant<int, G::gstart(c, g_.value)>{}, nL, dv_next, ri_next);
      });
      sfor<0, NS>([&](auto s_) {
        constexpr int s = s_.value;
        if constexpr (16 * s + 15 > c) A[G::off(s) + c] = nL[s];
      });
    });
    VEC_MARK("zero_upper");
    VEC_TMARK(4);
    // keep only the strict lower triangle of Lt (unit diagonal implied)
    sfor<0, NS>([&](auto s_) {
      constexpr int s = s_.value;
      const int r = row_of(s, l);
      sfor<16 * s, G::len(s)>([&](auto c_) {
        constexpr int c = c_.value;
        A[G::off(s) + c] = (c >= r) ? 0.0 : A[G::off(s) + c];
      });
    });
    // 1/d of this lane's rows
    sfor<0, NS>([&](auto s_) { idg[s_.value] = rec[grp][rrow[s_.value]][RI]; });

    // forward substitution x <- Lt^{-1} x (unit lower) for NV right-hand
    // sides, one column step at a time
    auto fwd_step = [&](auto c_, auto& x) {
      constexpr int c = decltype(c_)::value;
      constexpr int NV = std::extent<std::remove_reference_t<decltype(x)>, 0>::value;
      constexpr int sc = c / 16;
      constexpr int lc = G::lane_of(c);
      // x[v][row] += (x[v][c] broadcast from its owner) * (-Lt[row][c])
      // (A holds -Lt) for the slots holding rows below c.  Slots go in
      // decreasing order: the source x[v][sc] may share a register with the
      // accumulator of slot sc, which must then be the last one updated.
      constexpr int b = (c + 1) / 16;
      if constexpr (b < NS) {
        constexpr int NSL = NS - b;
        double acc[NV][NSL], src[NV], mul[NSL];
        sfor<0, NV>([&](auto v_) {
          src[v_.value] = x[v_.value][sc];
          sfor<0, NSL>([&](auto j_) { acc[v_.value][j_.value] = x[v_.value][NS - 1 - j_.value]; });
        });
        sfor<0, NSL>([&](auto j_) { mul[j_.value] = A[G::off(NS - 1 - j_.value) + c]; });
        dpp_fmac<NV, NSL, lc, lc, lc, lc>(acc, src, mul);
        sfor<0, NV>([&](auto v_) {
          sfor<0, NSL>([&](auto j_) { x[v_.value][NS - 1 - j_.value] = acc[v_.value][j_.value]; });
        });
      }
    };
    auto fwd = [&](auto& x) { sfor<0, K>([&](auto c_) { fwd_step(c_, x); }); };

    // ---------------- ut = Lt^{-T} e_last via Lt in LDS ----------------
    VEC_MARK("backsolve");
    VEC_TMARK(6);
    // Row r of Lt goes to Lp[r(r-1)/2 + c] for every column c < len(slot):
    // entries at c >= r (zeros) run into the rows after r, at smaller
    // columns.  Slots are stored in increasing row order and columns in
    // decreasing order, so every such spill-over is overwritten later by the
    // entry that belongs there (row r >= 1 spills into row r' > r at a
    // column at least r smaller, never within the same store); rows >= K and
    // row 0 write a sink.  No address arithmetic or select per entry.
    if constexpr (!kLik && !kRowBack) {
      sfor<0, NS>([&](auto s_) {
        constexpr int s = s_.value;
        double* __restrict__ dst = &Lp[grp][lrow_base[s]];
        sfor<0, G::len(s)>([&](auto cc_) {
          constexpr int c = G::len(s) - 1 - cc_.value;
          dst[c] = A[G::off(s) + c];
          // the order matters across lanes, which the compiler cannot see:
          // no reordering or pairing of these stores
          asm volatile("" ::: "memory");
        });
      });
    }
    double uu[NS];
    sfor<0, NS>([&](auto s_) { uu[s_.value] = (row_of(s_.value, l) == K - 1) ? 1.0 : 0.0; });
    wave_lds_fence();
    // Lt[r][row] for step r (0 where row >= r), read PF steps ahead: a
    // static offset from the lane's column base (entries at row >= r lie
    // inside Lp and are masked)
    auto lrow = [&](auto r_, double(&lv)[NS]) {
      constexpr int r = decltype(r_)::value;
      sfor<0, NS>([&](auto s_) {
        constexpr int s = s_.value;
        const double* __restrict__ src = &Lp[grp][lcol_base[s]];
        if constexpr (r > 0 && 16 * s + 15 < r) {
          // every row of the slot lies below r
          lv[s] = src[r * (r - 1) / 2];
        } else if constexpr (r > 0 && 16 * s < r) {
          const double v = src[r * (r - 1) / 2];
          lv[s] = (row_of(s, l) < r) ? v : 0.0;
        } else {
          lv[s] = 0.0;
        }
      });
    };
    constexpr int PF = (K < 3) ? K : 3;
    // one step of x <- Lt^{-T} x at row r = K - 1 - x_ (Lt[r][.] prefetched
    // PF steps ahead into the ring lvq)
    auto back_step = [&](auto x_, double(&lvq)[PF][NS], double(&xv)[NS]) {
      constexpr int x = decltype(x_)::value;
      constexpr int r = K - 1 - x;
      constexpr int sr = r / 16;
      constexpr int lr = G::lane_of(r);
      double lv[NS];
      sfor<0, NS>([&](auto s_) { lv[s_.value] = lvq[x % PF][s_.value]; });
      if constexpr (r - PF >= 0) lrow(std::integral_constant<int, r - PF>{}, lvq[x % PF]);
      // xv[row] += (xv[r] broadcast from its owner) * (-Lt[r][row]) for the
      // slots holding rows above r (Lp holds -Lt); the source may share a
      // register with the accumulator of slot sr, the last one updated
      if constexpr (r > 0) {
        constexpr int NSL = (r - 1) / 16 + 1;
        double acc[1][NSL], src[1] = {xv[sr]}, mul[NSL];
        sfor<0, NSL>([&](auto j_) {
          acc[0][j_.value] = xv[j_.value];
          mul[j_.value] = lv[j_.value];
        });
        dpp_fmac<1, NSL, lr>(acc, src, mul);
        sfor<0, NSL>([&](auto j_) { xv[j_.value] = acc[0][j_.value]; });
      }
    };
    auto back_prefetch = [&](auto& lvq) {
      if constexpr (!kRowBack)
        sfor<0, PF>([&](auto x_) { lrow(std::integral_constant<int, K - 1 - x_.value>{}, lvq[x_.value]); });
    };
    // Row-oriented step x of the same substitution (no copy of Lt): row
    // a = K - 2 - x gets xv[a] += sum_{r > a} (-Lt[r][a]) xv[r], the sum over
    // the lanes' rows from the factor in registers (upper entries are 0, so
    // no masks), then one 16-lane sum; the owner of row a adds it.
    auto back_step_rows = [&](auto x_, double(&xv)[NS]) {
      constexpr int a = K - 2 - decltype(x_)::value;
      if constexpr (a >= 0) {
        constexpr int b = (a + 1) / 16;  // slots holding rows > a
        double t = 0.0;
        sfor<b, NS>([&](auto s_) { t = __builtin_fma(A[G::off(s_.value) + a], xv[s_.value], t); });
        t = row_allreduce(t);
        constexpr int sa = a / 16;
        xv[sa] = (l == G::lane_of(a)) ? xv[sa] + t : xv[sa];
      }
    };
    if constexpr (kLik) {
      fwd(rhs);
    } else {
      double lvq[PF][NS];
      back_prefetch(lvq);
      // The back substitution (latency bound: one broadcast per step) runs
      // interleaved with the independent forward substitution of y and X.
      sfor<0, K>([&](auto x_) {
        if constexpr (kRowBack)
          back_step_rows(x_, uu);
        else
          back_step(x_, lvq, uu);
        fwd_step(x_, rhs);
      });
      // rhs = Lt^{-1} (y, X);  uu = Lt^{-T} e_last (u = uu / sqrt(d_last))
      if constexpr (kDeriv) {
        sfor<0, NS>([&](auto s_) {
          constexpr int s = s_.value;
          rec[grp][rrow[s]][RU] = uu[s];  // 0 for rows >= K
        });
        wave_lds_fence();
      }
    }
    if constexpr (kWts) {
      // uu = (-b, 1): the kriging weights of the neighbours in rows 0..q-1
      // (NNarray columns 1..q), zero for missing neighbours
      if (active) {
        double* __restrict__ wrow = a.rows_out + (i - a.i0) * (int64_t)(m + 1);
        sfor<0, NS>([&](auto s_) {
          constexpr int s = s_.value;
          const int r = row_of(s, l);
          if (r < m) wrow[r] = (r < q) ? -uu[s] : 0.0;
          if (r == K - 1) wrow[m] = log(vself * inv_sigma2);
        });
      }
    }

    if (more) fetch_vals(inext, idn, zv, yv, xv);  // next neighbourhood, in flight until the next gather
    VEC_MARK("phase2");
    VEC_TMARK(7);
    // ---------------- phase 2: g_rho = dSigma/drho * u (row layout) ----------------
    // g[a] = sum_b D_ab u_b for this lane's rows a: the pair factor comes
    // from sfv (static offsets off the diagonal block, the zero slot on the
    // diagonal), u_b and z_b are uniform reads, one column ahead of use.
    // Pairs with a padding row have exp(-h) = 0 and add nothing.
    // Adjoint: the back substitution alpha = Lt^{-T} D^{-1} yt (= Sigma^{-1} r)
    // runs interleaved, one step per column.
    double gr[NG][NS];
    double al[NS];
    if constexpr (kDeriv) {
    int base_a[NS];
    double zrow[NS][4];
    sfor<0, NS>([&](auto s_) {
      constexpr int s = s_.value;
      const int a = row_of(s, l);
      base_a[s] = qrow_base[s];
      if constexpr ((NG == 2 && !kTwoF) || kRecomp) {
#pragma unroll
        for (int k = 0; k < 4; ++k) zrow[s][k] = rec[grp][rrow[s]][RZ + k];
      }
#pragma unroll
      for (int g = 0; g < NG; ++g) gr[g][s] = 0.0;
    });
    auto col_load = [&](auto b_, double& ub, double(&zb)[4], double(&Sv)[NS], double(&Tv)[NS]) {
      constexpr int b = decltype(b_)::value;
      constexpr int CB = b * (b + 1) / 2;
      ub = rec[grp][b][RU];
      if constexpr ((NG == 2 && !kTwoF) || kRecomp) {
#pragma unroll
        for (int k = 0; k < 4; ++k) zb[k] = rec[grp][b][RZ + k];
      }
      if constexpr (!kRecomp) sfor<0, NS>([&](auto s_) {
        constexpr int s = s_.value;
        const int a = row_of(s, l);
        int idx;
        if constexpr (b < 16 * s)
          idx = base_a[s] + b;
        else if constexpr (b >= 16 * (s + 1))
          idx = a + CB;
        else
          idx = (b <= a) ? base_a[s] + b : a + CB;
        if constexpr (kTwoF) {
          // only the last slot holds rows >= K, whose indices pass the sink
          if constexpr (s == NS - 1 && K < 16 * NS) idx = idx < NQ ? idx : NQ;
          Sv[s] = sfv[grp][2 * idx];
          Tv[s] = sfv[grp][2 * idx + 1];
        } else {
          Sv[s] = sfv[grp][idx];
        }
      });
    };
    // pair factor of (row of slot s, column b) again, as in phase 1 (the
    // diagonal has h2 = 0 and padding rows exp(-h) = 0: both add 0)
    auto recompute = [&](const double(&zb)[4], double(&Sv)[NS]) {
      sfor<0, NS>([&](auto s_) {
        constexpr int s = s_.value;
        double h2 = kH2Floor;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double dz = zrow[s][k] - zb[k];
          h2 = __builtin_fma(dz, dz, h2);
        }
        double hh, hi;
        dist_from_sq(h2, hh, hi);
        const double x = fmax(-hh, -800.0);
        const double nn = rint(x * kInvLn2x64);
        const int in = (int)nn;
        const double T = exptab[in & 63];
        double r = __builtin_fma(-nn, kLn2d64Hi, x);
        r = __builtin_fma(-nn, kLn2d64Lo, r);
        double qq = __builtin_fma(r, 1.0 / 120.0, 1.0 / 24.0);
        qq = __builtin_fma(qq, r, 1.0 / 6.0);
        qq = __builtin_fma(qq, r, 0.5);
        qq = __builtin_fma(qq, r, 1.0);
        qq *= r;
        const double sE = ldexp(__builtin_fma(T, qq, T), in >> 6);
        const double sF = sE * __builtin_fma(cf.a1, hh, __builtin_fma(cf.a2, hi, cf.a0));
        Sv[s] = (NG == 1) ? sF * (h2 - kH2Floor) * cf.ir[0] : sF;
      });
    };
    // g_rho[row] += dSigma/drho (row, b) u_b for this lane's rows
    auto accumulate_col = [&](double ub, const double(&zb)[4], const double(&Sv)[NS],
                              const double(&Tv)[NS]) {
      sfor<0, NS>([&](auto s_) {
        constexpr int s = s_.value;
        if constexpr (kTwoF) {
          gr[0][s] = __builtin_fma(Sv[s], ub, gr[0][s]);
          gr[1][s] = __builtin_fma(Tv[s], ub, gr[1][s]);
        } else if constexpr (NG == 1) {
          // stored directly as dSigma/drho for the isotropic family
          gr[0][s] = __builtin_fma(Sv[s], ub, gr[0][s]);
        } else {
          const double d0 = zrow[s][0] - zb[0];
          double h2s = d0 * d0;
#pragma unroll
          for (int k = 1; k < 3; ++k) {
            const double dz = zrow[s][k] - zb[k];
            h2s = __builtin_fma(dz, dz, h2s);
          }
          const double dt = zrow[s][3] - zb[3];
          const double Su = Sv[s] * ub;
          gr[0][s] = __builtin_fma(Su, h2s, gr[0][s]);
          gr[1][s] = __builtin_fma(Su, dt * dt, gr[1][s]);
        }
      });
    };
    if constexpr (kRecomp && K > 41) {
      // Large neighbourhoods: a runtime loop over the columns keeps the
      // code small (the pair factors come from the coordinates, nothing is
      // indexed by register); the adjoint's back substitution runs first.
      if constexpr (kAdj) {
        sfor<0, NS>([&](auto s_) { al[s_.value] = rhs[0][s_.value] * idg[s_.value]; });
        sfor<0, K>([&](auto x_) { back_step_rows(x_, al); });
      }
      double ubn = rec[grp][0][RU], zbn[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) zbn[k] = rec[grp][0][RZ + k];
      for (int b = 0; b < K; ++b) {
        const double ub = ubn;
        double zb[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) zb[k] = zbn[k];
        const int bn = (b + 1 < K) ? b + 1 : b;
        ubn = rec[grp][bn][RU];
#pragma unroll
        for (int k = 0; k < 4; ++k) zbn[k] = rec[grp][bn][RZ + k];
        double Sv[NS], Tv[NS];
        recompute(zb, Sv);
        accumulate_col(ub, zb, Sv, Tv);
      }
    } else {
      double alq[PF][NS];
      if constexpr (kAdj) {
        sfor<0, NS>([&](auto s_) { al[s_.value] = rhs[0][s_.value] * idg[s_.value]; });
        back_prefetch(alq);
      }
      double ubn, zbn[4], Svn[NS], Tvn[NS];
      col_load(std::integral_constant<int, 0>{}, ubn, zbn, Svn, Tvn);
      sfor<0, K>([&](auto b_) {
        constexpr int b = b_.value;
        if constexpr (kAdj) {
          if constexpr (kRowBack)
            back_step_rows(b_, al);
          else
            back_step(b_, alq, al);
        }
        double ub = ubn, zb[4], Sv[NS], Tv[NS];
#pragma unroll
        for (int k = 0; k < 4; ++k) zb[k] = zbn[k];
        sfor<0, NS>([&](auto s_) {
          Sv[s_.value] = Svn[s_.value];
          Tv[s_.value] = Tvn[s_.value];
        });
        if constexpr (b + 1 < K)
          col_load(std::integral_constant<int, b + 1>{}, ubn, zbn, Svn, Tvn);
        if constexpr (kRecomp) recompute(zb, Sv);
        accumulate_col(ub, zb, Sv, Tv);
      });
    }
    if constexpr (NG == 2) {
      sfor<0, NS>([&](auto s_) {
        gr[0][s_.value] *= cf.ir[0];
        gr[1][s_.value] *= cf.ir[1];
      });
    }
    }  // kDeriv

    if constexpr (kFull) {
    VEC_MARK("w_solve");
    VEC_TMARK(8);
    // ---------------- w = L^{-1} (dSigma_j u) ----------------
    // range parameters: g_rho from phase 2; tau2: dSigma = sigma2 I.  In the
    // Lt form wt_j = Lt^{-1} dSigma_j uu, and w_j[l] = wt_j[l] / sqrt(d_l d_q).
    double w[NR][NS];
    sfor<0, NS>([&](auto s_) {
      constexpr int s = s_.value;
#pragma unroll
      for (int g = 0; g < NG; ++g) w[g][s] = gr[g][s];
      w[NG][s] = uu[s];
    });
    fwd(w);
    sfor<0, NS>([&](auto s_) { w[NG][s_.value] *= cf.sigma2; });

    VEC_MARK("sums");
    VEC_TMARK(9);
    // ---------------- per-neighbourhood sums ----------------
    // Sums over rows l < q in the Lt form: Sy_j = sum wt_j yt / d_l (times
    // 1/sqrt(d_q) later), SX_j likewise, G_jk = sum wt_j wt_k / d_l (times 1/d_q).
    double part[NPART];
    sfor<0, NPART>([&](auto e_) { part[e_.value] = 0.0; });
    sfor<0, NS>([&](auto s_) {
      constexpr int s = s_.value;
      const double keep = (row_of(s, l) < K - 1) ? idg[s] : 0.0;
      double ws[NR];
      sfor<0, NR>([&](auto j_) { ws[j_.value] = keep * w[j_.value][s]; });
      sfor<0, NR>([&](auto j_) {
        part[j_.value] = __builtin_fma(ws[j_.value], rhs[0][s], part[j_.value]);
      });
      sfor<0, NR>([&](auto j_) {
        sfor<0, PC>([&](auto t_) {
          constexpr int e = NR + j_.value * PC + t_.value;
          part[e] = __builtin_fma(ws[j_.value], rhs[1 + t_.value][s], part[e]);
        });
      });
      sfor<0, NR>([&](auto j_) {
        constexpr int j = j_.value;
        sfor<j, NR>([&](auto k_) {
          constexpr int k = k_.value;
          constexpr int e = NR + NR * PC + (j * (2 * NR - j + 1)) / 2 + (k - j);
          part[e] = __builtin_fma(ws[j], w[k][s], part[e]);
        });
      });
    });
    sfor<0, NPART>([&](auto e_) { part[e_.value] = row_allreduce(part[e_.value]); });

    VEC_MARK("accumulate");
    VEC_TMARK(10);
    if (active && l == LS) {
      // back from the Lt form to the quantities of the Cholesky factor L:
      // Liy_q = yt_q / sqrt(d_q), w_j[q] = wt_j[q] / d_q, Sy_j, SX_j carry
      // 1/sqrt(d_q), G_jk carries 1/d_q
      const double iq = idg[SS];
      const double sq = rsqrt_refined(vself);
      const double Lyq = rhs[0][SS] * sq;
      bool nonfinite = !(__builtin_isfinite(Lyq));
      sfor<0, PC>([&](auto t_) { nonfinite |= !(__builtin_isfinite(rhs[1 + t_.value][SS])); });
      // parameter j: 0 -> sigma2 (w = e_last / sigma2), j >= 1 -> w[j - 1]
      auto wq = [&](auto j_) -> double {
        constexpr int j = decltype(j_)::value;
        if constexpr (j == 0) return inv_sigma2; else return w[j - 1][SS] * iq;
      };
      auto Sy = [&](auto j_) -> double {
        constexpr int j = decltype(j_)::value;
        if constexpr (j == 0) return 0.0; else return part[j - 1] * sq;
      };
      auto SX = [&](auto j_, auto t_) -> double {
        constexpr int j = decltype(j_)::value, t = decltype(t_)::value;
        if constexpr (j == 0) return 0.0; else return part[NR + (j - 1) * PC + t] * sq;
      };
      auto Gjk = [&](auto j_, auto k_) -> double {
        constexpr int j = decltype(j_)::value, k = decltype(k_)::value;
        if constexpr (j == 0 || k == 0) {
          return 0.0;
        } else {
          constexpr int a = (j < k ? j : k) - 1, b = (j < k ? k : j) - 1;
          return part[NR + NR * PC + (a * (2 * NR - a + 1)) / 2 + (b - a)] * iq;
        }
      };
      auto LXq = [&](auto t_) -> double { return rhs[1 + decltype(t_)::value][SS] * sq; };
      double* ac = acc[grp];
      int ex;
      vprod[grp][0] = frexp(vprod[grp][0] * vself, &ex);
      vprod[grp][1] += (double)ex;
      ac[1] += Lyq * Lyq;
      constexpr int oXSX = 2, oySX = oXSX + PC * PC, odl = oySX + PC, ody = odl + P,
                    odX = ody + P, odyX = odX + P * PC * PC, oin = odyX + P * PC;
      sfor<0, PC>([&](auto s_) {
        sfor<0, PC>([&](auto t_) { ac[oXSX + s_.value * PC + t_.value] += LXq(s_) * LXq(t_); });
        ac[oySX + s_.value] += Lyq * LXq(s_);
      });
      sfor<0, P>([&](auto j_) {
        constexpr int j = j_.value;
        const double wj = wq(j_);
        ac[odl + j] += wj;
        ac[ody + j] += -2.0 * Lyq * Sy(j_) - wj * Lyq * Lyq;
        sfor<0, PC>([&](auto s_) {
          sfor<0, PC>([&](auto t_) {
            ac[odX + (j * PC + s_.value) * PC + t_.value] +=
                -(SX(j_, s_) * LXq(t_) + LXq(s_) * SX(j_, t_)) - wj * LXq(s_) * LXq(t_);
          });
          ac[odyX + j * PC + s_.value] += -Sy(j_) * LXq(s_) - Lyq * SX(j_, s_) - wj * Lyq * LXq(s_);
        });
        sfor<0, P>([&](auto k_) { ac[oin + j * P + k_.value] += Gjk(j_, k_) + 0.5 * wj * wq(k_); });
      });
      static_assert(oin + P * P == NRAW, "raw layout");
      const int flags = (notpd ? 1 : 0) | (nonfinite ? 4 : 0);
      if (flags) {
        atomicOr(&status[0], flags);
        atomicMin(&status[1], (int32_t)i);
      }
    }
    } else if constexpr (kAdj) {
    VEC_MARK("adjoint");
    // ---------------- reverse-mode gradient ----------------
    // With v = d_q and e = yt_q (conditional variance and residual of the
    // self row), the neighbourhood's term -1/2 (log v + e^2 / v) has
    // derivative, for dSigma_j,
    //   -1/2 [ (ut' dSigma_j ut) (1 + e^2/v) / v - 2 e (alpha' dSigma_j ut) / v ],
    // where ut = Lt^{-T} e_last and alpha = Sigma^{-1} r.  Range parameters
    // use g_j = dSigma_j ut from phase 2, tau2 uses g = sigma2 ut and sigma2
    // reduces to -1/2 (1 - e^2/v) / sigma2 (Sigma ut = v e_last).
    constexpr int ND = 2 * NG + 2;
    double dots[ND];
    sfor<0, ND>([&](auto e_) { dots[e_.value] = 0.0; });
    sfor<0, NS>([&](auto s_) {
      constexpr int s = s_.value;
      sfor<0, NG>([&](auto g_) {
        constexpr int g = g_.value;
        dots[2 * g] = __builtin_fma(uu[s], gr[g][s], dots[2 * g]);
        dots[2 * g + 1] = __builtin_fma(al[s], gr[g][s], dots[2 * g + 1]);
      });
      dots[2 * NG] = __builtin_fma(uu[s], uu[s], dots[2 * NG]);
      dots[2 * NG + 1] = __builtin_fma(al[s], uu[s], dots[2 * NG + 1]);
    });
    sfor<0, ND>([&](auto e_) { dots[e_.value] = row_allreduce(dots[e_.value]); });
    if (active && l == LS) {
      const double iv = idg[SS];
      const double e = rhs[0][SS];
      const double e2v = e * e * iv;
      const double c1 = (1.0 + e2v) * iv, c2 = 2.0 * e * iv;
      const bool nonfinite = !(__builtin_isfinite(e2v));
      double* ac = acc[grp];
      int ex;
      vprod[grp][0] = frexp(vprod[grp][0] * vself, &ex);
      vprod[grp][1] += (double)ex;
      ac[1] += e2v;
      ac[2] += -0.5 * (1.0 - e2v) * inv_sigma2;
      sfor<0, NG>([&](auto g_) {
        constexpr int g = g_.value;
        ac[3 + g] += -0.5 * (dots[2 * g] * c1 - c2 * dots[2 * g + 1]);
      });
      ac[1 + P] += -0.5 * cf.sigma2 * (dots[2 * NG] * c1 - c2 * dots[2 * NG + 1]);
      static_assert(2 + P == NRAW, "adjoint layout");
      const int flags = (notpd ? 1 : 0) | (nonfinite ? 4 : 0);
      if (flags) {
        atomicOr(&status[0], flags);
        atomicMin(&status[1], (int32_t)i);
      }
    }
    } else {
    VEC_MARK("loglik");
    // ---------------- sums of Algorithm 1 ----------------
    if (active && l == LS) {
      const double sq = rsqrt_refined(vself);
      const double Lyq = rhs[0][SS] * sq;
      double LXq[PC];
      bool nonfinite = !(__builtin_isfinite(Lyq));
      sfor<0, PC>([&](auto t_) {
        LXq[t_.value] = rhs[1 + t_.value][SS] * sq;
        nonfinite |= !(__builtin_isfinite(LXq[t_.value]));
      });
      double* ac = acc[grp];
      int ex;
      vprod[grp][0] = frexp(vprod[grp][0] * vself, &ex);
      vprod[grp][1] += (double)ex;
      ac[1] += Lyq * Lyq;
      sfor<0, PC>([&](auto s_) {
        sfor<0, PC>([&](auto t_) { ac[2 + s_.value * PC + t_.value] += LXq[s_.value] * LXq[t_.value]; });
        ac[2 + PC * PC + s_.value] += Lyq * LXq[s_.value];
      });
      static_assert(2 + PC * PC + PC == NRAW, "loglik layout");
      const int flags = (notpd ? 1 : 0) | (nonfinite ? 4 : 0);
      if (flags) {
        atomicOr(&status[0], flags);
        atomicMin(&status[1], (int32_t)i);
      }
    }
    }
    VEC_TMARK(11);
    badnn = badnn || badidx;
    if (active && (badnn || badval)) {
      atomicOr(&status[0], (badnn ? 2 : 0) | (badval ? 4 : 0));
      atomicMin(&status[1], (int32_t)i);
    }
    sfor<0, NS>([&](auto s_) { idc[s_.value] = idn[s_.value]; });
    badc = badn;
    skipc = skipn;
    wave_lds_fence();
  }
  if constexpr (BATCH) {
    flush(a.partials + (a.batch.row0 + tile) * NRAW);
    tile = grab();
  } else {
    break;
  }
  }  // tiles
  VEC_TFLUSH;
  if constexpr (!BATCH) flush(a.partials + (int64_t)blockIdx.x * NRAW);
}

// Host-side launcher of one instantiation.
template <int K, int PC, int NG, int MODE, bool BATCH>
hipError_t launch_sums(int grid, hipStream_t stream, const SumsArgs& args) {
  hipLaunchKernelGGL((sums_kernel<K, PC, NG, MODE, BATCH>), dim3(grid), dim3(kThreads), 0, stream,
                     args);
  return hipGetLastError();
}

// Resident workgroups per CU of one instantiation (0 on error).
template <int K, int PC, int NG, int MODE, bool BATCH>
int resident_sums() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sums_kernel<K, PC, NG, MODE, BATCH>,
                                                   kThreads, 0) != hipSuccess)
    return 0;
  return nb;
}

using launch_fn = hipError_t (*)(int, hipStream_t, const SumsArgs&);
using resident_fn = int (*)();

// Explicit instantiation of one K and p: both range layouts, the three
// modes of the single-problem kernel and the batched sums kernel.
#define VECCHIA_LAUNCH_SIG(K, PC, NG, MODE, B) \
  hipError_t launch_sums<K, PC, NG, MODE, B>(int, hipStream_t, const SumsArgs&)
#define VECCHIA_RESIDENT_SIG(K, PC, NG, MODE, B) int resident_sums<K, PC, NG, MODE, B>()
#define VECCHIA_FOR_NG(X, K, PC, NG) \
  X(K, PC, NG, 0, false);            \
  X(K, PC, NG, 1, false);            \
  X(K, PC, NG, 2, false);            \
  X(K, PC, NG, 3, false);            \
  X(K, PC, NG, 0, true)
#define VECCHIA_FOR_MODES(X, K, PC) \
  VECCHIA_FOR_NG(X, K, PC, 1);      \
  VECCHIA_FOR_NG(X, K, PC, 2)
// single-problem modes only (sizes without a batched class)
#define VECCHIA_FOR_SINGLE(X, K, PC) \
  X(K, PC, 1, 0, false);             \
  X(K, PC, 1, 1, false);             \
  X(K, PC, 1, 2, false);             \
  X(K, PC, 1, 3, false);             \
  X(K, PC, 2, 0, false);             \
  X(K, PC, 2, 1, false);             \
  X(K, PC, 2, 2, false);             \
  X(K, PC, 2, 3, false)

// single-problem modes of one range layout
#define VECCHIA_FOR_NG_SINGLE(X, K, PC, NG) \
  X(K, PC, NG, 0, false);                   \
  X(K, PC, NG, 1, false);                   \
  X(K, PC, NG, 2, false);                   \
  X(K, PC, NG, 3, false)

// Instantiated K values of the single-problem kernel (K >= m + 1 is padded
// with rows that decouple) and the sizes of the batched classes.
constexpr int kNumK = 6;
constexpr int kKs[kNumK] = {11, 21, 31, 35, 41, 61};
constexpr int kNumBatchK = 4;
constexpr int kBatchKs[kNumBatchK] = {11, 21, 31, 41};

}  // namespace vecchia

// Wave-per-neighbourhood Vecchia sums, FP64, gfx950: the kernel for what the
// 16-lane fused kernel does not hold in registers --
//   * one range per coordinate (Section 4.3, Eq. 6 with rho_1..rho_d; the
//     high-dimensional regression setting of Section 4.2): P = d + 2
//     derivative directions and an O(P^2) information block;
//   * neighbourhoods of more than 41 observations (m up to 63);
//   * grouped Vecchia (Section 2.1): the conditional density of a block of
//     g consecutive observations given a conditioning set of c earlier ones.
// A single observation is a block of one whose conditioning set is its
// NNarray row, so one code path serves all three.
//
// A workgroup is one wave; it loops over blocks i0 + blockIdx.x,
// + gridDim.x, ... and keeps its sums in LDS (lane l owns the entries
// e = l (mod 64)), written once to partials[blockIdx.x][nraw] at the end.
//
// Per block, local order: the c conditioning observations, then the g block
// members (k = c + g <= 64 rows):
//   gather      scaled coordinates z / rho (zero-padded to DMAX), y, X.
//   covariance  pairs spread over the lanes: Sigma transposed into the upper
//               triangle of A, the pair factor F_ab = -sigma2 f'(h)/h into the
//               lower one (dSigma_ab/drho = F_ab s^2 / rho, s the scaled
//               coordinate difference of that range).
//   Cholesky    Sigma = L L' in registers, lane r holding row r; column
//               entries broadcast with readlane; L' written back to A.
//   U           U = L^-T E_B, the block's g unit vectors (back substitution,
//               lanes = rows, the g columns side by side).
//   G_j         G_j = dSigma_j U for every range j (lanes = rows; the column
//               loop split between the two half-waves when k <= 32).
//   solves      L^-1 applied to y, X, every G_j and U (one column per lane;
//               with at most six columns, lanes = rows).
//   Gram        products of the solved columns over the conditioning rows.
//   sums        with W_j = L^-1 dSigma_j U (W_sigma2 = E_B / sigma2,
//               W_tau2 = sigma2 L^-1 U), z = L^-1 y, Z = L^-1 X and b, b'
//               running over the block rows:
//                 logdet   += sum_b log L_bb^2,  ySy += sum_b z_b^2, ...
//                 dlogdet_j += sum_b W_j[b, b]
//                 dySy_j   += -2 sum_b z_b (W_j' z)_<c,b - sum_bb' z_b W_j[b, b'] z_b'
//                 ainfo_jk += sum_b (W_j' W_k)_<c,bb + 1/2 sum_bb' W_j[b, b'] W_k[b, b']
//               (the differences between the joint terms over the
//               neighbourhood and those over the conditioning set, in the
//               factor's coordinates; one block row gives the fused kernel's
//               single-observation terms).
#include <math.h>

#include <type_traits>

#include "vecchia.h"
#include "vecchia_wave.hpp"

namespace vecchia_wave {
namespace {

constexpr int kLanes = 64;

// Offsets (in doubles) of the per-workgroup LDS regions.
struct Layout {
  int SA, SZ, SV, NR, P, nraw;
  int oA, oZ, oV, oG, oAcc, oDinv, oInvRho, oTri, oDesc, total;
};

// kmax: neighbourhood rows; dmax: coordinate slots per row (the slots
// d..dmax-1 hold zeros); R range parameters; gmax: largest block.  NR is
// the number of solved columns of the largest block.
__host__ __device__ inline Layout layout_of(int kmax, int dmax, int R, int p, int gmax) {
  Layout L;
  L.SA = kmax + 1;  // odd: column accesses by lane hit distinct banks
  L.SZ = dmax + 2;  // even: rows start 16-byte aligned
  L.SV = kmax + 1;
  L.P = R + 2;
  L.NR = 1 + p + (R + 1) * gmax;  // y, X, G_j (g columns each), U (g columns)
  L.nraw = 2 + p * p + p + L.P * (2 + p * p + p) + L.P * L.P;
  const int T = kmax > L.NR ? kmax : L.NR;  // largest triangle enumerated
  int o = 0;
  L.oA = o;
  o += kmax * L.SA;
  L.oZ = o;
  o += kmax * L.SZ;
  L.oV = o;
  o += (L.NR + 1) * L.SV;  // row NR: a sink for the stores of unused coordinates
  L.oG = o;
  o += L.NR * L.NR;
  L.oAcc = o;
  o += L.nraw;
  L.oDinv = o;
  o += kmax;
  L.oInvRho = o;
  o += kMaxD;
  L.oTri = o;
  o += (T * (T + 1) / 2 + 1) / 2;
  L.oDesc = o;  // one int32 per raw entry
  o += (L.nraw + 1) / 2;
  L.total = o;
  return L;
}

// LDS operations of one wave complete in program order, and a workgroup is
// one wave: ordering them needs only a compiler fence.
__device__ __forceinline__ void wave_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// The value itself, hidden from the optimiser at this point of the block
// loop: comparisons of a per-coordinate or per-column index with it are then
// made where they are used instead of being hoisted out of the loop and kept
// live (as scalar masks) across every step.
__device__ __forceinline__ int opaque_v(int x) {
  asm volatile("" : "+v"(x));
  return x;
}
__device__ __forceinline__ int opaque_s(int x) {
  asm volatile("" : "+s"(x));
  return x;
}

__device__ __forceinline__ double readlane_d(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 1/sqrt(x): hardware estimate y0 and one second-order Newton correction,
// y = y0 (1 + e/2 + 3e^2/8) with e = 1 - x y0^2.
__device__ __forceinline__ double rsqrt_nr(double x) {
  const double y0 = __builtin_amdgcn_rsq(x);
  const double e = fma(-(x * y0), y0, 1.0);
  return fma(y0 * e, fma(0.375, e, 0.5), y0);
}

// Profiling builds only (-DVECCHIA_WAVE_TIMING, with a device array
// unsigned long long wave_cycles[16] defined before this file is compiled):
// shader-clock cycles of each step of the block loop, summed over waves.
#ifdef VECCHIA_WAVE_TIMING
#define WAVE_TDECL                     \
  unsigned long long tsec_[9] = {};    \
  unsigned long long t_last_ = clock64();
#define WAVE_TMARK(idx)                          \
  do {                                           \
    __builtin_amdgcn_sched_barrier(0);           \
    const unsigned long long t_ = clock64();     \
    tsec_[idx] += t_ - t_last_;                  \
    t_last_ = t_;                                \
    __builtin_amdgcn_sched_barrier(0);           \
  } while (0)
#define WAVE_TFLUSH \
  if (lane == 0)    \
    for (int k_ = 0; k_ < 9; ++k_) atomicAdd(&wave_cycles[k_], tsec_[k_]);
#else
#define WAVE_TDECL
#define WAVE_TMARK(idx)
#define WAVE_TFLUSH
#endif

__device__ __forceinline__ void flag(int32_t* status, int f, int64_t i) {
  atomicOr(&status[0], f);
  atomicMin(&status[1], (int32_t)i);
}

// A (KMAX x SA): Sigma transposed in the upper triangle (A[c][r] = Sigma_rc,
// c <= r) until the factorisation, then L transposed there (A[c][r] =
// L_rc); the strict lower triangle holds the pair factors (A[r][c] = F_rc).
template <int KMAX, int DMAX, int GMAX>
__global__ __launch_bounds__(kLanes) void wave_kernel(const WaveArgs a) {
  extern __shared__ double lds[];
  const int lane = threadIdx.x;
  const int m = a.m, d = a.d, p = a.p, nu = a.nu, R = a.R;
  const bool per_coord = (a.family == VEC_FAMILY_ANISO);
  const bool grouped = (a.block_start != nullptr);
  const Layout Ly = layout_of(KMAX, DMAX, R, p, grouped ? a.gmax : 1);
  const int SA = Ly.SA, SZ = Ly.SZ, SV = Ly.SV, P = Ly.P, nraw = Ly.nraw;
  double* __restrict__ A = lds + Ly.oA;
  double* __restrict__ Z = lds + Ly.oZ;
  double* __restrict__ V = lds + Ly.oV;
  double* __restrict__ G = lds + Ly.oG;
  double* __restrict__ acc = lds + Ly.oAcc;
  double* __restrict__ dinv = lds + Ly.oDinv;
  double* __restrict__ invrho = lds + Ly.oInvRho;
  int32_t* __restrict__ tri = reinterpret_cast<int32_t*>(lds + Ly.oTri);
  int32_t* __restrict__ edesc = reinterpret_cast<int32_t*>(lds + Ly.oDesc);

  const double sigma2 = a.covparms[0], tau2 = a.covparms[R + 1];
  // range parameter of coordinate k
  auto grp = [&](int k) {
    return per_coord ? k : ((a.family == VEC_FAMILY_SPACETIME && k >= a.nspace) ? 1 : 0);
  };
  // tri[r (r + 1) / 2 + c] = (r, c), c <= r: the pair enumeration of the
  // covariance pairs and of the Gram pairs
  const int T = KMAX > Ly.NR ? KMAX : Ly.NR;
  for (int r = lane; r < T; r += kLanes)
    for (int c = 0; c <= r; ++c) tri[r * (r + 1) / 2 + c] = r | (c << 16);
  for (int k = lane; k < kMaxD; k += kLanes) invrho[k] = (k < d) ? 1.0 / a.covparms[1 + grp(k)] : 0.0;
  // edesc[e]: what raw entry e is -- kind (0 logdet, 1 ySy, 2 XSX, 3 ySX,
  // 4 dlogdet, 5 dySy, 6 dXSX, 7 dySX, 8 ainfo) | j << 4 | k << 10 |
  // s << 16 | s2 << 18 (parameters j, k; covariates s, s2)
  for (int e = lane; e < nraw; e += kLanes) {
    acc[e] = 0.0;
    int o = e, kind, j = 0, k = 0, s1 = 0, s2 = 0;
    if (o == 0) {
      kind = 0;
    } else if (o == 1) {
      kind = 1;
    } else if ((o -= 2) < p * p) {
      kind = 2, s1 = o / p, s2 = o % p;
    } else if ((o -= p * p) < p) {
      kind = 3, s1 = o;
    } else if ((o -= p) < P) {
      kind = 4, j = o;
    } else if ((o -= P) < P) {
      kind = 5, j = o;
    } else if ((o -= P) < P * p * p) {
      kind = 6, j = o / (p * p), s1 = (o % (p * p)) / p, s2 = o % p;
    } else if ((o -= P * p * p) < P * p) {
      kind = 7, j = o / p, s1 = o % p;
    } else {
      o -= P * p;
      kind = 8, j = o / P, k = o % P;
    }
    edesc[e] = kind | (j << 4) | (k << 10) | (s1 << 16) | (s2 << 18);
  }
  wave_fence();
  WAVE_TDECL

  for (int64_t u = a.i0 + blockIdx.x; u < a.i1; u += gridDim.x) {
    // ---- the block: first member, size g, conditioning set (c entries)
    int64_t first, cbase = 0;
    int c, g;
    const int32_t* row = nullptr;
    if (grouped) {
      first = a.block_start[u];
      const int64_t last = a.block_start[u + 1];
      cbase = a.cond_start[u];
      const int64_t cend = a.cond_start[u + 1];
      const bool ok = first >= 0 && last > first && last - first <= a.gmax && last <= a.n &&
                      cbase >= 0 && cend >= cbase && cend <= a.ncond && cend - cbase <= m &&
                      (cend - cbase) + (last - first) <= KMAX;
      if (!ok) {  // the same values in every lane
        if (lane == 0) flag(a.status, VEC_FLAG_BADNN, first > 0 ? first : 0);
        continue;
      }
      g = (GMAX == 1) ? 1 : (int)(last - first);  // GMAX == 1 serves gmax <= 1 only
      c = (int)(cend - cbase);
    } else {
      first = u;
      g = 1;
      c = (int)(u < m ? u : m);
      row = a.NN + u * (int64_t)(m + 1);
    }
    const int kk = c + g;
    bool bad = false;
    int64_t src = first + (lane - c);
    if (lane < c) {
      const int32_t j = grouped ? a.cond[cbase + lane] : row[1 + lane];
      bad = (j < 0 || (int64_t)j >= first);
      src = bad ? 0 : j;
    } else if (!grouped && lane == c) {
      bad = (row[0] != (int32_t)u);
    }
    if (__ballot(bad) != 0ull) {
      if (lane == 0) flag(a.status, VEC_FLAG_BADNN, first);
      continue;
    }

    WAVE_TMARK(0);
    // ---- gather: scaled coordinates (zero-padded to DMAX), y, X
    if (lane < kk) {
      const double* zs = a.locs + src * d;
      const int dd = opaque_s(d);
      double z[DMAX];
#pragma unroll
      for (int k = 0; k < DMAX; ++k) z[k] = (k < dd) ? zs[k] : 0.0;
#pragma unroll
      for (int k = 0; k < DMAX; ++k) Z[lane * SZ + k] = z[k] * invrho[k];
      V[lane] = a.y[src];
      for (int t = 0; t < p; ++t) V[(1 + t) * SV + lane] = a.X[src * p + t];
    }
    wave_fence();

    WAVE_TMARK(1);
    // ---- covariance (transposed, upper) and pair factors (lower)
    const int npair = kk * (kk + 1) / 2;
    for (int e = lane; e < npair; e += kLanes) {
      const int t = tri[e];
      const int r = t & 0xffff, cc = t >> 16;
      const double* zr = Z + r * SZ;
      const double* zc = Z + cc * SZ;
      double h2 = 0.0;
#pragma unroll
      for (int k = 0; k < DMAX; ++k) {
        const double dz = zr[k] - zc[k];
        h2 = fma(dz, dz, h2);
      }
      const double h = sqrt(h2);
      const double E = exp(-h);
      double f, F;
      if (nu == 0) {
        f = E;
        F = (h > 0.0) ? E / h : 0.0;
      } else if (nu == 1) {
        f = (1.0 + h) * E;
        F = E;
      } else {
        f = (1.0 + h + h * h / 3.0) * E;
        F = (1.0 + h) * E / 3.0;
      }
      A[cc * SA + r] = sigma2 * (f + (r == cc ? tau2 : 0.0));
      if (r != cc) A[r * SA + cc] = sigma2 * F;
    }
    wave_fence();

    WAVE_TMARK(2);
    // ---- Cholesky in registers: lane r holds row r; the entries of column
    // cc are broadcast lane by lane (readlane into scalar registers).  Rows
    // and columns >= kk carry garbage that never reaches a row < kk
    // (right-looking updates only flow to larger indices).
    bool notpd = false;
    {
      double Ar[KMAX];
#pragma unroll
      for (int cc = 0; cc < KMAX; ++cc) Ar[cc] = A[cc * SA + (lane < KMAX ? lane : 0)];
      // Column cc's entries are broadcast CG at a time, each group's
      // readlanes ahead of its updates.  Up to 48 rows the next pivot is
      // taken, and its inverse square root started, right after the first
      // group's updates, so that chain overlaps the rest of the column (at 64
      // rows that longer code measured slower).
      constexpr int CG = 4;
      auto update = [&](double lrc, int s0) {
        double b[CG];
#pragma unroll
        for (int q = 0; q < CG; ++q)
          if (s0 + q < KMAX) b[q] = readlane_d(lrc, s0 + q);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < CG; ++q)
          if (s0 + q < KMAX) Ar[s0 + q] = fma(-lrc, b[q], Ar[s0 + q]);
      };
      if constexpr (KMAX <= 48) {
        double piv = readlane_d(Ar[0], 0);
        double inv = rsqrt_nr(piv);
        double myinv = 0.0;  // lane cc keeps 1 / L_cc,cc
#pragma unroll
        for (int cc = 0; cc < KMAX; ++cc) {
          if (cc < kk) {  // columns past the neighbourhood are skipped whole
            notpd = notpd || !(piv > 0.0);
            const double lrc = Ar[cc] * inv;
            Ar[cc] = lrc;
            myinv = (lane == cc) ? inv : myinv;
#pragma unroll
            for (int s0 = cc + 1; s0 < KMAX; s0 += CG) {
              update(lrc, s0);
              if (s0 == cc + 1) {
                piv = readlane_d(Ar[cc + 1], cc + 1);
                inv = rsqrt_nr(piv);
              }
              __builtin_amdgcn_sched_barrier(0);
            }
          }
        }
        if (lane < kk) dinv[lane] = myinv;
      } else {
#pragma unroll
        for (int cc = 0; cc < KMAX; ++cc) {
          if (cc < kk) {
            const double piv = readlane_d(Ar[cc], cc);
            notpd = notpd || !(piv > 0.0);
            const double inv = rsqrt_nr(piv);
            const double lrc = Ar[cc] * inv;
            Ar[cc] = lrc;
            if (lane == 0) dinv[cc] = inv;
#pragma unroll
            for (int s0 = cc + 1; s0 < KMAX; s0 += CG) {
              update(lrc, s0);
              __builtin_amdgcn_sched_barrier(0);
            }
          }
        }
      }
      // L transposed into the upper triangle: A[cc][r] = L_r,cc for cc <= r
      if (lane < kk) {
        const int ln = opaque_v(lane);
#pragma unroll
        for (int cc = 0; cc < KMAX; ++cc)
          if (cc <= ln) A[cc * SA + lane] = Ar[cc];
      }
    }
    if (notpd) {
      if (lane == 0) flag(a.status, VEC_FLAG_NOTPD, first);
      continue;
    }
    wave_fence();

    // solved columns of this block: y, X, then g per range, then g for U
    const int NR = 1 + p + (R + 1) * g;
    const int oU = 1 + p + R * g;

    WAVE_TMARK(3);
    // ---- U = L^-T E_B by back substitution (lane r holds U[r][t]); the
    // next column's pivot factor and L entries are loaded one step ahead
    {
      double ub[GMAX];
#pragma unroll
      for (int t = 0; t < GMAX; ++t) ub[t] = (lane == c + t) ? 1.0 : 0.0;
      const int lrow = lane < KMAX ? lane : 0;
      double dcn = dinv[kk - 1];
      double lcn = A[lrow * SA + kk - 1];  // L[kk - 1][lane], used where lane < kk - 1
      for (int col = kk - 1; col >= 0; --col) {
        const double dc = dcn, lcl = lcn;
        if (col > 0) {
          dcn = dinv[col - 1];
          lcn = A[lrow * SA + col - 1];
        }
#pragma unroll
        for (int t = 0; t < GMAX; ++t) {
          if (t < g) {
            const double uc = readlane_d(ub[t], col) * dc;
            const double upd = fma(-lcl, uc, ub[t]);
            ub[t] = (lane < col) ? upd : ((lane == col) ? uc : ub[t]);
          }
        }
      }
      if (lane < kk) {
#pragma unroll
        for (int t = 0; t < GMAX; ++t)
          if (t < g) V[(oU + t) * SV + lane] = ub[t];
      }
    }
    wave_fence();

    WAVE_TMARK(4);
    // ---- G_j[r][t] = sum_b F_rb s_j(r, b)^2 U[b][t] / rho_j
    {
      constexpr int H = kLanes / KMAX > 1 ? 2 : 1;  // column halves
      const int r = lane % KMAX, half = (H == 2) ? lane / (kLanes / 2) : 0;
      const bool rowl = (H == 2) ? (lane % (kLanes / 2)) == r : true;
      const int hb = (kk + H - 1) / H;
      const int b0 = half * hb, b1 = (b0 + hb < kk) ? b0 + hb : kk;
      double zr[DMAX], gs[DMAX][GMAX];
#pragma unroll
      for (int k = 0; k < DMAX; ++k) {
        zr[k] = Z[r * SZ + k];
#pragma unroll
        for (int t = 0; t < GMAX; ++t) gs[k][t] = 0.0;
      }
      if (r < kk && rowl) {
        // with many coordinates the next column's are loaded while this
        // one's are used
        constexpr bool kAhead = DMAX >= 8;
        double zn[DMAX];
        if constexpr (kAhead) {
#pragma unroll
          for (int k = 0; k < DMAX; ++k) zn[k] = Z[b0 * SZ + k];
        }
        // the pair factor and U entries of the next column are loaded one
        // step ahead (the last step re-reads its own)
        auto pairF = [&](int b) { return A[(b < r ? r : b) * SA + (b < r ? b : r)]; };
        double Fn = pairF(b0), un[GMAX];
#pragma unroll
        for (int t = 0; t < GMAX; ++t) un[t] = V[(oU + t) * SV + b0];
        for (int b = b0; b < b1; ++b) {
          const int bn = (b + 1 < b1) ? b + 1 : b;
          double zb[DMAX];
          if constexpr (kAhead) {
#pragma unroll
            for (int k = 0; k < DMAX; ++k) zb[k] = zn[k];
#pragma unroll
            for (int k = 0; k < DMAX; ++k) zn[k] = Z[bn * SZ + k];
          } else {
#pragma unroll
            for (int k = 0; k < DMAX; ++k) zb[k] = Z[b * SZ + k];
          }
          // b == r adds nothing: its coordinate differences are exactly 0
          const double F = (b == r) ? 0.0 : Fn;
          double cb[GMAX];
#pragma unroll
          for (int t = 0; t < GMAX; ++t) cb[t] = (t < g) ? F * un[t] : 0.0;
          Fn = pairF(bn);
#pragma unroll
          for (int t = 0; t < GMAX; ++t) un[t] = V[(oU + t) * SV + bn];
#pragma unroll
          for (int k = 0; k < DMAX; ++k) {
            const double s = zr[k] - zb[k];
            const double s2 = s * s;
#pragma unroll
            for (int t = 0; t < GMAX; ++t) gs[k][t] = fma(cb[t], s2, gs[k][t]);
          }
        }
      }
      if constexpr (H == 2) {
#pragma unroll
        for (int k = 0; k < DMAX; ++k)
#pragma unroll
          for (int t = 0; t < GMAX; ++t) gs[k][t] += __shfl_xor(gs[k][t], kLanes / 2);
      }
      if (half == 0 && r < kk && rowl) {
#pragma unroll
        for (int t = 0; t < GMAX; ++t) {
          if (t >= g) continue;
          // every 1 / rho_k is read before the first store
          double ir[DMAX];
#pragma unroll
          for (int k = 0; k < DMAX; ++k) ir[k] = invrho[k];
          if (per_coord) {
            // coordinates past d (zero sums) go to the sink row
            const int dd = opaque_s(d);
#pragma unroll
            for (int k = 0; k < DMAX; ++k) {
              const int row = (k < dd) ? 1 + p + k * g + t : Ly.NR;
              V[row * SV + r] = gs[k][t] * ir[k];
            }
          } else {  // coordinates sharing a range add up (past d: zeros)
            // coordinates before ns have the first range
            const int ns = opaque_s(a.family == VEC_FAMILY_SPACETIME ? a.nspace : DMAX);
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int k = 0; k < DMAX; ++k) {
              const double v = gs[k][t] * ir[k];
              const bool first = k < ns;
              s0 += first ? v : 0.0;
              s1 += first ? 0.0 : v;
            }
            V[(1 + p + t) * SV + r] = s0;
            if (R > 1) V[(1 + p + g + t) * SV + r] = s1;
          }
        }
      }
    }
    wave_fence();

    WAVE_TMARK(5);
    // ---- L^-1 applied to every solved column.  With few columns (y, X and
    // the derivative columns of one observation with one or two ranges) lanes
    // are rows and the columns advance together, one factor column per step
    // (right-looking); otherwise one column per lane.
    auto row_solve = [&](auto nm_) {
      constexpr int NM = decltype(nm_)::value;
      const int lr = lane < KMAX ? lane : 0;
      const int nr = opaque_s(NR);
      double xv[NM];
#pragma unroll
      for (int j = 0; j < NM; ++j) xv[j] = (j < nr) ? V[j * SV + lr] : 0.0;
      // the next step's pivot factor and L entries are loaded one step ahead
      double dcn = dinv[0], lcn = A[lr];  // L[lane][0]
      for (int col = 0; col < kk; ++col) {
        const double dc = dcn, lcl = lcn;
        if (col + 1 < kk) {
          dcn = dinv[col + 1];
          lcn = A[(col + 1) * SA + lr];  // L[lane][col + 1] where lane > col + 1
        }
        double xc[NM];
#pragma unroll
        for (int j = 0; j < NM; ++j) xc[j] = readlane_d(xv[j], col);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < NM; ++j) {
          const double x = xc[j] * dc;
          const double upd = fma(-lcl, x, xv[j]);
          xv[j] = (lane > col) ? upd : ((lane == col) ? x : xv[j]);
        }
      }
      if (lane < kk) {
#pragma unroll
        for (int j = 0; j < NM; ++j)
          if (j < nr) V[j * SV + lane] = xv[j];
      }
    };
    if (NR <= 4) {
      row_solve(std::integral_constant<int, 4>{});
    } else if (NR <= 6) {
      row_solve(std::integral_constant<int, 6>{});
    } else if (lane < NR) {  // one column per lane
      double* __restrict__ vj = V + lane * SV;
      double x[KMAX];
      // rows in blocks of 8, a block skipped as a whole once past kk (rows
      // kk.. of a computed block read stale LDS and are not stored)
#pragma unroll
      for (int rb = 0; rb < KMAX; rb += 8) {
        if (rb < kk) {
#pragma unroll
          for (int r = rb; r < rb + 8; ++r) {
            double s = vj[r];
#pragma unroll
            for (int cc = 0; cc < r; ++cc) s = fma(-A[cc * SA + r], x[cc], s);
            x[r] = s * dinv[r];
            if (r < kk) vj[r] = x[r];
          }
        }
      }
    }
    wave_fence();

    WAVE_TMARK(6);
    // ---- Gram matrix of the solved columns over the conditioning rows
    const int ng = NR * (NR + 1) / 2;
    for (int e = lane; e < ng; e += kLanes) {
      const int t = tri[e];
      const int j = t & 0xffff, k = t >> 16;
      const double* vj = V + j * SV;
      const double* vk = V + k * SV;
      double s0 = 0.0, s1 = 0.0;
      int l = 0;
      for (; l + 1 < c; l += 2) {
        s0 = fma(vj[l], vk[l], s0);
        s1 = fma(vj[l + 1], vk[l + 1], s1);
      }
      if (l < c) s0 = fma(vj[l], vk[l], s0);
      G[j * NR + k] = s0 + s1;
      G[k * NR + j] = s0 + s1;
    }
    wave_fence();

    WAVE_TMARK(7);
    // ---- the block rows' terms, entry by entry (lane-owned accumulators)
    bool finite = true;
    for (int t = 0; t < g; ++t) {
      finite = finite && isfinite(V[c + t]);
      for (int s = 0; s < p; ++s) finite = finite && isfinite(V[(1 + s) * SV + c + t]);
    }
    if (!finite) {
      if (lane == 0) flag(a.status, VEC_FLAG_NONFINITE, first);
      continue;
    }
    // parameter j: 0 = sigma2, 1..R = ranges, P - 1 = tau2; column of
    // parameter j >= 1 for block row t
    auto col = [&](int j, int t) { return j == P - 1 ? oU + t : 1 + p + (j - 1) * g + t; };
    auto cf = [&](int j) { return j == P - 1 ? sigma2 : 1.0; };
    auto zB = [&](int t) { return V[c + t]; };
    auto XB = [&](int t, int s) { return V[(1 + s) * SV + c + t]; };
    // W_j[c + rr][t]
    auto wq = [&](int j, int rr, int t) {
      return j == 0 ? (rr == t ? 1.0 / sigma2 : 0.0) : cf(j) * V[col(j, t) * SV + c + rr];
    };
    auto Sy = [&](int j, int t) { return j == 0 ? 0.0 : cf(j) * G[col(j, t) * NR]; };
    auto SX = [&](int j, int t, int s) {
      return j == 0 ? 0.0 : cf(j) * G[col(j, t) * NR + 1 + s];
    };
    auto GG = [&](int j, int k, int t) {
      return (j == 0 || k == 0) ? 0.0 : cf(j) * cf(k) * G[col(j, t) * NR + col(k, t)];
    };
    for (int e = lane; e < nraw; e += kLanes) {
      const int code = edesc[e];
      const int kind = code & 15, j = (code >> 4) & 63, k = (code >> 10) & 63,
                s = (code >> 16) & 3, s2 = (code >> 18) & 3;
      double v = 0.0;
      switch (kind) {
        case 0:
          for (int t = 0; t < g; ++t) v += -2.0 * log(dinv[c + t]);
          break;
        case 1:
          for (int t = 0; t < g; ++t) v += zB(t) * zB(t);
          break;
        case 2:
          for (int t = 0; t < g; ++t) v += XB(t, s) * XB(t, s2);
          break;
        case 3:
          for (int t = 0; t < g; ++t) v += zB(t) * XB(t, s);
          break;
        case 4:
          for (int t = 0; t < g; ++t) v += wq(j, t, t);
          break;
        case 5:
          for (int t = 0; t < g; ++t) {
            v += -2.0 * zB(t) * Sy(j, t);
            for (int rr = 0; rr < g; ++rr) v -= zB(rr) * wq(j, rr, t) * zB(t);
          }
          break;
        case 6:
          for (int t = 0; t < g; ++t) {
            v -= XB(t, s) * SX(j, t, s2) + SX(j, t, s) * XB(t, s2);
            for (int rr = 0; rr < g; ++rr) v -= XB(rr, s) * wq(j, rr, t) * XB(t, s2);
          }
          break;
        case 7:
          for (int t = 0; t < g; ++t) {
            v -= zB(t) * SX(j, t, s) + Sy(j, t) * XB(t, s);
            for (int rr = 0; rr < g; ++rr) v -= zB(rr) * wq(j, rr, t) * XB(t, s);
          }
          break;
        default:
          for (int t = 0; t < g; ++t) {
            v += GG(j, k, t);
            for (int rr = 0; rr < g; ++rr) v += 0.5 * wq(j, rr, t) * wq(k, rr, t);
          }
          break;
      }
      acc[e] += v;
    }
    wave_fence();
    WAVE_TMARK(8);
  }
  WAVE_TFLUSH
  double* out = a.partials + (int64_t)blockIdx.x * nraw;
  for (int e = lane; e < nraw; e += kLanes) out[e] = acc[e];
}

template <int KMAX, int DMAX, int GMAX>
hipError_t launch_t(const WaveArgs& a, int grid, hipStream_t st) {
  const Layout L = layout_of(KMAX, DMAX, a.R, a.p, a.block_start ? a.gmax : 1);
  const size_t bytes = (size_t)L.total * sizeof(double);
  if (bytes > 65536) {
    const hipError_t e =
        hipFuncSetAttribute(reinterpret_cast<const void*>(wave_kernel<KMAX, DMAX, GMAX>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((wave_kernel<KMAX, DMAX, GMAX>), dim3(grid), dim3(kLanes), bytes, st, a);
  return hipGetLastError();
}

template <int KMAX>
hipError_t launch_k(const WaveArgs& a, int grid, hipStream_t st) {
  if (a.block_start && a.gmax > 4) return launch_t<KMAX, 4, 8>(a, grid, st);
  if (a.block_start && a.gmax > 2) return launch_t<KMAX, 4, 4>(a, grid, st);
  if (a.block_start && a.gmax > 1) return launch_t<KMAX, 4, 2>(a, grid, st);
  if (a.d <= 4) return launch_t<KMAX, 4, 1>(a, grid, st);
  if (a.d <= 8) return launch_t<KMAX, 8, 1>(a, grid, st);
  if (a.d <= 16) return launch_t<KMAX, 16, 1>(a, grid, st);
  if (a.d <= 20) return launch_t<KMAX, 20, 1>(a, grid, st);
  return launch_t<KMAX, 32, 1>(a, grid, st);
}

}  // namespace

int wave_grid(int64_t total) {
  if (total <= 0) return 0;
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      ncu = v;
  }
  const int64_t cap = (int64_t)ncu * 8;
  return (int)(total < cap ? total : cap);
}

hipError_t launch_wave(const WaveArgs& a, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  const int kmax = a.block_start ? a.m + a.gmax : a.m + 1;
  if (kmax <= 16) return launch_k<16>(a, grid, st);
  if (kmax <= 32) return launch_k<32>(a, grid, st);
  if (kmax <= 48) return launch_k<48>(a, grid, st);
  return launch_k<64>(a, grid, st);
}

}  // namespace vecchia_wave

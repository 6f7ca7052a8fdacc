// Per-neighbourhood Vecchia sums for covariances with one range per
// coordinate (Section 4.3, Eq. 6 with rho_1..rho_d; the high-dimensional
// regression setting of Section 4.2), FP64, gfx950.
//
// With P = d + 2 covariance parameters the per-neighbourhood state (P
// derivative directions, a P x P information block, nraw = O(P^2) sums)
// no longer fits the 16-lane register layout of the fused kernel, so this
// kernel gives each neighbourhood a whole wave and keeps the matrices in
// LDS.  A workgroup is one wave; it loops over observations i0 + blockIdx.x,
// + gridDim.x, ... and keeps its sums in LDS (each lane owns the entries
// e = lane (mod 64)), written once to partials[blockIdx.x][nraw] at the end.
//
// Steps per neighbourhood (local order: the q neighbours, then i last):
//   gather      scaled coordinates z_k / rho_k, y, X into LDS.
//   covariance  lower triangle of Sigma (pairs spread over the lanes); the
//               upper triangle keeps the pair factor F_ab = -sigma2 f'(h)/h,
//               so that dSigma_ab/drho_k = F_ab s_k^2 / rho_k with
//               s_k = (z_ak - z_bk) / rho_k.
//   Cholesky    right-looking, in place; trailing updates spread over lanes.
//   u           u = L^-T e_q (back substitution, lanes = rows).
//   g_k         g_k = dSigma/drho_k u for every range k: lanes = rows, the
//               column loop split between the two half-waves at m + 1 <= 32.
//   solves      L^-1 applied to y, X, g_1..g_d and u (one column per lane).
//   Gram        G = V_<q' V_<q over all solved columns (pairs over lanes).
//   sums        with w_j = L^-1 dSigma_j u (w_sigma2 = e_q / sigma2,
//               w_tau2 = sigma2 L^-1 u), Sy_j, SX_j and G_jk from the Gram
//               matrix, the self row adds the same terms as the fused kernel:
//                 logdet += log L_qq^2, ySy += Liy_q^2, ...,
//                 ainfo_jk += G_jk + w_j[q] w_k[q] / 2.
#include <math.h>

#include "vecchia.h"
#include "vecchia_aniso.hpp"

namespace vecchia_aniso {
namespace {

constexpr int kLanes = 64;

// Offsets (in doubles) of the per-workgroup LDS regions.
struct Layout {
  int SA, SZ, SV, NR, P, nraw;
  int oA, oZ, oV, oG, oAcc, oDinv, oInvRho, oTri, oIdx, total;
};

__host__ __device__ inline Layout layout_of(int kmax, int d, int p) {
  Layout L;
  L.SA = kmax + 2;                    // rows of Sigma / L
  L.SZ = (d % 2 == 0) ? d + 1 : d;    // rows of scaled coordinates (odd stride)
  L.SV = kmax + 1;                    // solved columns
  L.P = d + 2;
  L.NR = 1 + p + d + 1;               // y, X, g_1..g_d, u
  L.nraw = 2 + p * p + p + L.P * (2 + p * p + p) + L.P * L.P;
  const int T = kmax > L.NR ? kmax : L.NR;  // largest triangle enumerated
  int o = 0;
  L.oA = o;
  o += kmax * L.SA;
  L.oZ = o;
  o += kmax * L.SZ;
  L.oV = o;
  o += L.NR * L.SV;
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
  L.oIdx = o;
  o += (kmax + 1) / 2;
  L.total = o;
  return L;
}

__device__ __forceinline__ double readlane_d(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int KMAX, int DMAX>
__global__ __launch_bounds__(kLanes) void aniso_kernel(const AnisoArgs a) {
  extern __shared__ double lds[];
  const int lane = threadIdx.x;
  const int m = a.m, d = a.d, p = a.p, nu = a.nu;
  const Layout Ly = layout_of(KMAX, d, p);
  const int SA = Ly.SA, SZ = Ly.SZ, SV = Ly.SV, NR = Ly.NR, P = Ly.P, nraw = Ly.nraw;
  double* __restrict__ A = lds + Ly.oA;
  double* __restrict__ Z = lds + Ly.oZ;
  double* __restrict__ V = lds + Ly.oV;
  double* __restrict__ G = lds + Ly.oG;
  double* __restrict__ acc = lds + Ly.oAcc;
  double* __restrict__ dinv = lds + Ly.oDinv;
  double* __restrict__ invrho = lds + Ly.oInvRho;
  int32_t* __restrict__ tri = reinterpret_cast<int32_t*>(lds + Ly.oTri);
  int32_t* __restrict__ idx = reinterpret_cast<int32_t*>(lds + Ly.oIdx);

  const double sigma2 = a.covparms[0], tau2 = a.covparms[d + 1];
  // tri[r (r + 1) / 2 + c] = (r, c), c <= r: the pair enumeration of every
  // triangle below (covariance pairs, trailing updates, Gram pairs)
  const int T = KMAX > NR ? KMAX : NR;
  for (int r = lane; r < T; r += kLanes)
    for (int c = 0; c <= r; ++c) tri[r * (r + 1) / 2 + c] = r | (c << 16);
  for (int k = lane; k < d; k += kLanes) invrho[k] = 1.0 / a.covparms[1 + k];
  for (int e = lane; e < nraw; e += kLanes) acc[e] = 0.0;
  __syncthreads();

  for (int64_t i = a.i0 + blockIdx.x; i < a.i1; i += gridDim.x) {
    const int q = (int)(i < m ? i : m), kk = q + 1;
    const int32_t* row = a.NN + i * (int64_t)(m + 1);
    bool bad = false;
    if (lane < q) {
      const int32_t j = row[1 + lane];
      bad = (j < 0 || (int64_t)j >= i);
      idx[lane] = bad ? 0 : j;
    } else if (lane == q) {
      bad = (row[0] != (int32_t)i);
      idx[q] = (int32_t)i;
    }
    if (__ballot(bad) != 0ull) {
      if (lane == 0) {
        atomicOr(&a.status[0], VEC_FLAG_BADNN);
        atomicMin(&a.status[1], (int32_t)i);
      }
      __syncthreads();
      continue;
    }
    __syncthreads();

    // ---- gather: scaled coordinates, y, X (lanes = local rows)
    if (lane < kk) {
      const int64_t s = idx[lane];
      const double* zs = a.locs + s * d;
      for (int k = 0; k < d; ++k) Z[lane * SZ + k] = zs[k] * invrho[k];
      V[lane] = a.y[s];
      for (int t = 0; t < p; ++t) V[(1 + t) * SV + lane] = a.X[s * p + t];
    }
    __syncthreads();

    // ---- covariance (lower) and range-derivative pair factor (upper)
    const int npair = kk * (kk + 1) / 2;
    for (int e = lane; e < npair; e += kLanes) {
      const int t = tri[e];
      const int r = t & 0xffff, c = t >> 16;
      const double* zr = Z + r * SZ;
      const double* zc = Z + c * SZ;
      double h2 = 0.0;
      for (int k = 0; k < d; ++k) {
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
      A[r * SA + c] = sigma2 * (f + (r == c ? tau2 : 0.0));
      if (r != c) A[c * SA + r] = sigma2 * F;
    }
    __syncthreads();

    // ---- Cholesky, lower triangle in place; dinv[c] = 1 / L_cc
    bool notpd = false;
    for (int c = 0; c < kk; ++c) {
      const double piv = A[c * SA + c];
      if (!(piv > 0.0)) {  // the same value in every lane
        notpd = true;
        break;
      }
      const double inv = 1.0 / sqrt(piv);
      if (lane == 0) dinv[c] = inv;
      for (int r = c + 1 + lane; r < kk; r += kLanes) A[r * SA + c] *= inv;
      __syncthreads();
      const int nt = kk - 1 - c, ntri = nt * (nt + 1) / 2;
      for (int e = lane; e < ntri; e += kLanes) {
        const int t = tri[e];
        const int r = c + 1 + (t & 0xffff), s = c + 1 + (t >> 16);
        A[r * SA + s] = fma(-A[r * SA + c], A[s * SA + c], A[r * SA + s]);
      }
      __syncthreads();
    }
    if (notpd) {
      if (lane == 0) {
        atomicOr(&a.status[0], VEC_FLAG_NOTPD);
        atomicMin(&a.status[1], (int32_t)i);
      }
      __syncthreads();
      continue;
    }

    // ---- u = L^-T e_q by back substitution (lane r holds u_r)
    double ub = (lane == q) ? 1.0 : 0.0;
    for (int c = q; c >= 0; --c) {
      const double uc = readlane_d(ub, c) * dinv[c];
      if (lane < c)
        ub = fma(-A[c * SA + lane], uc, ub);
      else if (lane == c)
        ub = uc;
    }
    double* __restrict__ U = V + (NR - 1) * SV;
    if (lane < kk) U[lane] = ub;
    __syncthreads();

    // ---- g_k[r] = sum_b F_rb s_k(r, b)^2 u_b / rho_k
    {
      constexpr int H = kLanes / KMAX;  // column halves
      const int r = lane % KMAX, half = lane / KMAX;
      const int hb = (kk + H - 1) / H;
      const int b0 = half * hb, b1 = (b0 + hb < kk) ? b0 + hb : kk;
      double zr[DMAX], g[DMAX];
#pragma unroll
      for (int k = 0; k < DMAX; ++k) {
        zr[k] = (k < d && r < kk) ? Z[r * SZ + k] : 0.0;
        g[k] = 0.0;
      }
      if (r < kk) {
        for (int b = b0; b < b1; ++b) {
          if (b == r) continue;
          const int lo = b < r ? b : r, hi = b < r ? r : b;
          const double cb = A[lo * SA + hi] * U[b];
          const double* zb = Z + b * SZ;
#pragma unroll
          for (int k = 0; k < DMAX; ++k) {
            if (k < d) {
              const double s = zr[k] - zb[k];
              g[k] = fma(cb * s, s, g[k]);
            }
          }
        }
      }
      if constexpr (H == 2) {
#pragma unroll
        for (int k = 0; k < DMAX; ++k)
          if (k < d) g[k] += __shfl_xor(g[k], 32);
      }
      if (half == 0 && r < kk) {
#pragma unroll
        for (int k = 0; k < DMAX; ++k)
          if (k < d) V[(1 + p + k) * SV + r] = g[k] * invrho[k];
      }
    }
    __syncthreads();

    // ---- L^-1 applied to every column (one column per lane)
    if (lane < NR) {
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
            for (int c = 0; c < r; ++c) s = fma(-A[r * SA + c], x[c], s);
            x[r] = s * dinv[r];
            if (r < kk) vj[r] = x[r];
          }
        }
      }
    }
    __syncthreads();

    // ---- Gram matrix of the solved columns over the rows l < q
    const int ng = NR * (NR + 1) / 2;
    for (int e = lane; e < ng; e += kLanes) {
      const int t = tri[e];
      const int j = t & 0xffff, k = t >> 16;
      const double* vj = V + j * SV;
      const double* vk = V + k * SV;
      double s = 0.0;
      for (int l = 0; l < q; ++l) s = fma(vj[l], vk[l], s);
      G[j * NR + k] = s;
      G[k * NR + j] = s;
    }
    __syncthreads();

    // ---- the self row's terms, entry by entry (lane-owned accumulators)
    const double Lyq = V[q];
    bool finite = isfinite(Lyq);
    for (int t = 0; t < p; ++t) finite = finite && isfinite(V[(1 + t) * SV + q]);
    if (!finite) {
      if (lane == 0) {
        atomicOr(&a.status[0], VEC_FLAG_NONFINITE);
        atomicMin(&a.status[1], (int32_t)i);
      }
      __syncthreads();
      continue;
    }
    // parameter j: 0 = sigma2, 1..d = rho_j, P - 1 = tau2
    auto col = [&](int j) { return j == P - 1 ? NR - 1 : p + j; };
    auto cf = [&](int j) { return j == 0 ? 0.0 : (j == P - 1 ? sigma2 : 1.0); };
    auto wq = [&](int j) { return j == 0 ? 1.0 / sigma2 : cf(j) * V[col(j) * SV + q]; };
    auto Sy = [&](int j) { return j == 0 ? 0.0 : cf(j) * G[col(j) * NR]; };
    auto SX = [&](int j, int t) { return j == 0 ? 0.0 : cf(j) * G[col(j) * NR + 1 + t]; };
    auto Gjk = [&](int j, int k) {
      return (j == 0 || k == 0) ? 0.0 : cf(j) * cf(k) * G[col(j) * NR + col(k)];
    };
    auto LX = [&](int t) { return V[(1 + t) * SV + q]; };
    for (int e = lane; e < nraw; e += kLanes) {
      int o = e;
      double v;
      if (o == 0) {
        v = -2.0 * log(dinv[q]);
      } else if (o == 1) {
        v = Lyq * Lyq;
      } else if ((o -= 2) < p * p) {
        v = LX(o / p) * LX(o % p);
      } else if ((o -= p * p) < p) {
        v = Lyq * LX(o);
      } else if ((o -= p) < P) {
        v = wq(o);
      } else if ((o -= P) < P) {
        v = -2.0 * Lyq * Sy(o) - wq(o) * Lyq * Lyq;
      } else if ((o -= P) < P * p * p) {
        const int j = o / (p * p), st = o % (p * p), s = st / p, t = st % p;
        v = -(SX(j, s) * LX(t) + LX(s) * SX(j, t)) - wq(j) * LX(s) * LX(t);
      } else if ((o -= P * p * p) < P * p) {
        const int j = o / p, t = o % p;
        v = -Sy(j) * LX(t) - Lyq * SX(j, t) - wq(j) * Lyq * LX(t);
      } else {
        o -= P * p;
        const int j = o / P, k = o % P;
        v = Gjk(j, k) + 0.5 * wq(j) * wq(k);
      }
      acc[e] += v;
    }
    __syncthreads();
  }
  double* out = a.partials + (int64_t)blockIdx.x * nraw;
  for (int e = lane; e < nraw; e += kLanes) out[e] = acc[e];
}

template <int KMAX, int DMAX>
hipError_t launch_t(const AnisoArgs& a, int grid, hipStream_t st) {
  const Layout L = layout_of(KMAX, a.d, a.p);
  const size_t bytes = (size_t)L.total * sizeof(double);
  if (bytes > 65536) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(aniso_kernel<KMAX, DMAX>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)bytes);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((aniso_kernel<KMAX, DMAX>), dim3(grid), dim3(kLanes), bytes, st, a);
  return hipGetLastError();
}

}  // namespace

int aniso_grid(int64_t total) {
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

hipError_t launch_aniso(const AnisoArgs& a, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  const bool small = a.m + 1 <= 32;
  if (a.d <= 8) return small ? launch_t<32, 8>(a, grid, st) : launch_t<64, 8>(a, grid, st);
  if (a.d <= 16) return small ? launch_t<32, 16>(a, grid, st) : launch_t<64, 16>(a, grid, st);
  return small ? launch_t<32, 32>(a, grid, st) : launch_t<64, 32>(a, grid, st);
}

}  // namespace vecchia_aniso

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
//   gather    locsub/ysub/Xsub: coordinates pre-scaled by 1/rho, to LDS.
//   phase 1   covariance entries, one pair per lane per step with no idle
//             lanes: off-diagonal 16x16 blocks directly, and the two
//             triangular diagonal blocks of a slot pair folded into a
//             17-step loop (lane l takes row l's entry while u <= l, else
//             row 31-l's entry at column 32-u).
//   Cholesky  right-looking in registers; column c broadcast with
//             row_newbcast from its owner lane.
//   solves    Liy = L^-1 y, LiX = L^-1 X; L to LDS; u = L^-T e_last.
//   phase 2   g_rho = (dSigma/drho) u for each range parameter: pairs are
//             scheduled as a round-robin tournament (each round pairs every
//             row with a distinct partner), so the scatter g[a] += D u_b,
//             g[b] += D u_a is conflict-free LDS ds_add_f64 traffic; the
//             derivative entries are recomputed, never stored.
//   w         w_rho = L^-1 g_rho, w_tau2 = sigma2 L^-1 u, w_sigma2 =
//             e_last / sigma2 (dSigma/dsigma2 = Sigma / sigma2).
//   sums      with Sy_j = sum_{l<q} w_j[l] Liy[l], SX_j likewise,
//             G_jk = sum_{l<q} w_j[l] w_k[l] (one DPP all-reduce), the self
//             row gives
//               logdet += log v,  ySy += Liy_q^2, XSX += LiX_q LiX_q^T,
//               ySX += Liy_q LiX_q,  dlogdet_j += w_j[q],
//               dySy_j += -2 Liy_q Sy_j - w_j[q] Liy_q^2,
//               dXSX_j += -(SX_j LiX_q^T + LiX_q SX_j^T) - w_j[q] LiX_q LiX_q^T,
//               dySX_j += -Sy_j LiX_q - Liy_q SX_j - w_j[q] Liy_q LiX_q,
//               ainfo_jk += G_jk + w_j[q] w_k[q] / 2,
//             accumulated per group in LDS by the self row's lane.
// The per-workgroup sums go to partials[block][nraw]; a second kernel adds
// them in a fixed order, so results are deterministic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace vecchia {

constexpr int kGroupsPerBlock = 4;
constexpr int kThreads = 64;

// nu codes: 0 -> 1/2, 1 -> 3/2, 2 -> 5/2
constexpr int nraw_of(int p, int P) { return 2 + p * p + p + P * (2 + p * p + p) + P * P; }

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
  return __builtin_amdgcn_update_dpp(0.0, x, 0x150 + LANE, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
  return __builtin_amdgcn_update_dpp(0.0, x, CTRL, 0xF, 0xF, false);
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
  static constexpr int lane_of(int r) {
    return ((r / 16) & 1) ? 16 * (r / 16) + 15 - r : r - 16 * (r / 16);
  }
};

__device__ __forceinline__ int row_of(int s, int l) { return 16 * s + ((s & 1) ? 15 - l : l); }

// h = sqrt(h2) and 1/h, both 0 at h2 = 0.
__device__ __forceinline__ void dist_from_sq(double h2, double& h, double& hinv) {
  const bool pos = h2 > 0.0;
  const double r = rsqrt_refined(pos ? h2 : 1.0);
  h = pos ? h2 * r : 0.0;
  hinv = pos ? r : 0.0;
}

struct CovCoef {
  double sigma2, diag;  // sigma2, sigma2 * (1 + tau2)
  double c1, c2;        // f = (1 + c1 h + c2 h^2) e^-h
  double a0, a1, a2;    // -f'(h)/h = (a0 + a1 h + a2/h) e^-h
  double irk[4];        // per-coordinate 1/range
  double msk[4];        // 1 for coordinates of the second range group
  double ir[2];         // 1/range per group
};

template <int K, int PC, int NG>
__global__ __launch_bounds__(kThreads) void sums_kernel(
    const int m, const int d, const int nspace, const int nu, const double* __restrict__ locs,
    const int32_t* __restrict__ NN, const double* __restrict__ y, const double* __restrict__ X,
    const double* __restrict__ covparms, const int64_t i0, const int64_t i1,
    double* __restrict__ partials, int32_t* __restrict__ status) {
  using G = Geo<K>;
  constexpr int NS = G::NS;
  constexpr int KP = G::KP;
  constexpr int NL = G::NL;
  constexpr int P = NG + 2;   // sigma2, ranges, tau2
  constexpr int NR = NG + 1;  // parameters whose w has entries above the self row
  constexpr int NRAW = nraw_of(PC, P);
  constexpr int LPN = K * (K + 1) / 2;
  constexpr int SS = G::slot_of(K - 1);
  constexpr int LS = G::lane_of(K - 1);
  constexpr int NGR = NR * (NR + 1) / 2;
  constexpr int NPART = NR + NR * PC + NGR;

  __shared__ double zs[kGroupsPerBlock][KP][4];
  __shared__ double Lp[kGroupsPerBlock][LPN];
  __shared__ double uv[kGroupsPerBlock][KP];
  __shared__ double gv[kGroupsPerBlock][NG][KP];
  __shared__ double acc[kGroupsPerBlock][NRAW];

  const int l = threadIdx.x & 15;
  const int grp = threadIdx.x >> 4;

  CovCoef cf;
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
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const bool g1 = (NG == 2) && (k >= nspace);
    cf.irk[k] = g1 ? cf.ir[1] : cf.ir[0];
    cf.msk[k] = g1 ? 1.0 : 0.0;
  }
  const double inv_sigma2 = 1.0 / cf.sigma2;

  for (int e = threadIdx.x; e < kGroupsPerBlock * NRAW; e += kThreads) (&acc[0][0])[e] = 0.0;

  const int64_t total = i1 - i0;
  for (int64_t base = (int64_t)blockIdx.x * kGroupsPerBlock; base < total;
       base += (int64_t)gridDim.x * kGroupsPerBlock) {
    const bool active = base + grp < total;
    const int64_t i = i0 + (active ? base + grp : total - 1);
    const int q = (int)(i < (int64_t)m ? i : (int64_t)m);
    const int32_t* nnrow = NN + i * (int64_t)(m + 1);
    bool badnn = false;

    // ---------------- gather ----------------
    int kind[NS];  // 0 neighbour, 1 padding, 2 self, 3 beyond K
    double zo[NS][4];
    double rhs[1 + PC][NS];
    if (l == LS) badnn |= (nnrow[0] != (int32_t)i);
    sfor<0, NS>([&](auto s_) {
      constexpr int s = s_.value;
      const int r = row_of(s, l);
      int kd = 1;
      int64_t id = -1;
      if (r >= K) {
        kd = 3;
      } else if (r == K - 1) {
        kd = 2;
        id = i;
      } else if (r < q) {
        const int64_t j = nnrow[1 + r];
        if (j < 0 || j >= i) {
          badnn = true;
        } else {
          kd = 0;
          id = j;
        }
      }
      kind[s] = kd;
      const bool has = id >= 0;
      const int64_t ids = has ? id : i;  // always a valid row for the loads
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double v = (k < d) ? locs[ids * d + k] : 0.0;
        zo[s][k] = has ? v * cf.irk[k] : 0.0;
        zs[grp][r][k] = zo[s][k];
      }
      rhs[0][s] = has ? y[ids] : 0.0;
#pragma unroll
      for (int t = 0; t < PC; ++t) rhs[1 + t][s] = has ? X[ids * PC + t] : 0.0;
    });
    __syncthreads();

    // off-diagonal covariance of two scaled locations
    auto cov_off = [&](const double* za, const double* zb) -> double {
      double h2 = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double t = za[k] - zb[k];
        h2 = __builtin_fma(t, t, h2);
      }
      double h, hinv;
      dist_from_sq(h2, h, hinv);
      const double E = exp(-h);
      return cf.sigma2 * __builtin_fma(h, __builtin_fma(h, cf.c2, cf.c1), 1.0) * E;
    };

    // ---------------- phase 1: covariance ----------------
    double A[NL];
    sfor<0, NL>([&](auto e_) { A[e_.value] = 0.0; });
    bool realr[NS];
    sfor<0, NS>([&](auto s_) { realr[s_.value] = (kind[s_.value] == 0) || (kind[s_.value] == 2); });

    // off-diagonal 16x16 blocks: slot s rows x columns of block t < s
    sfor<1, NS>([&](auto s_) {
      constexpr int s = s_.value;
      sfor<0, s>([&](auto t_) {
        constexpr int t = t_.value;
        sfor<0, 16>([&](auto cc_) {
          constexpr int c = 16 * t + cc_.value;
          double zc[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) zc[k] = zs[grp][c][k];
          const double v = cov_off(zo[s], zc);
          A[G::off(s) + c] = (realr[s] && (c < q)) ? v : 0.0;
        });
      });
    });
    // diagonal blocks of slots (2t, 2t+1) folded into 17 steps
    sfor<0, NS / 2>([&](auto t_) {
      constexpr int s0 = 2 * t_.value;
      constexpr int s1 = s0 + 1;
      sfor<0, 17>([&](auto u_) {
        constexpr int u = u_.value;
        const bool first = (u <= l);
        const int c = first ? 16 * s0 + u : 16 * s1 + 16 - u;
        const int r = first ? row_of(s0, l) : row_of(s1, l);
        const bool rr = first ? realr[s0] : realr[s1];
        double zr[4], zc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          zr[k] = first ? zo[s0][k] : zo[s1][k];
          zc[k] = zs[grp][c][k];
        }
        const bool rc = (c < q) || (c == K - 1);
        const double off = cov_off(zr, zc);
        const double v = (c == r) ? (rr ? cf.diag : 1.0) : ((rr && rc) ? off : 0.0);
        if constexpr (u <= 15) A[G::off(s0) + 16 * s0 + u] = first ? v : A[G::off(s0) + 16 * s0 + u];
        if constexpr (u >= 1 && 16 * s1 + 16 - u < K)
          A[G::off(s1) + 16 * s1 + 16 - u] = first ? A[G::off(s1) + 16 * s1 + 16 - u] : v;
      });
    });
    // unpaired last slot (odd NS): its triangle directly
    if constexpr (NS & 1) {
      constexpr int s = NS - 1;
      sfor<0, G::len(s) - 16 * s>([&](auto u_) {
        constexpr int u = u_.value;
        constexpr int c = 16 * s + u;
        const int r = row_of(s, l);
        double zc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) zc[k] = zs[grp][c][k];
        const bool rc = (c < q) || (c == K - 1);
        const double off = cov_off(zo[s], zc);
        const double v = (c == r) ? (realr[s] ? cf.diag : 1.0) : ((realr[s] && rc) ? off : 0.0);
        A[G::off(s) + c] = (u <= l) ? v : 0.0;
      });
    }

    // ---------------- Cholesky (right-looking, in registers) ----------------
    double idg[NS];
    sfor<0, NS>([&](auto s_) { idg[s_.value] = 0.0; });
    bool notpd = false;
    double vself = 1.0;
    sfor<0, K>([&](auto c_) {
      constexpr int c = c_.value;
      constexpr int sc = c / 16;
      constexpr int lc = G::lane_of(c);
      const double dv = bcast<lc>(A[G::off(sc) + c]);
      notpd |= !(dv > 0.0);
      const double rs = rsqrt_refined(dv);
      const double pv = dv * rs;
      if constexpr (c == K - 1) vself = dv;
      sfor<0, NS>([&](auto s_) {
        constexpr int s = s_.value;
        if constexpr (16 * s + 15 >= c) {
          const int r = row_of(s, l);
          A[G::off(s) + c] = (r == c) ? pv : A[G::off(s) + c] * rs;
          idg[s] = (r == c) ? rs : idg[s];
        }
      });
      sfor<c + 1, K>([&](auto r_) {
        constexpr int r = r_.value;
        constexpr int sr = r / 16;
        constexpr int lr = G::lane_of(r);
        const double lrc = bcast<lr>(A[G::off(sr) + c]);
        sfor<0, NS>([&](auto s_) {
          constexpr int s = s_.value;
          if constexpr (16 * s + 15 >= r)
            A[G::off(s) + r] = __builtin_fma(-A[G::off(s) + c], lrc, A[G::off(s) + r]);
        });
      });
    });
    // keep only the strict lower triangle (diagonal lives in idg as 1/L_rr)
    sfor<0, NS>([&](auto s_) {
      constexpr int s = s_.value;
      const int r = row_of(s, l);
      sfor<16 * s, G::len(s)>([&](auto c_) {
        constexpr int c = c_.value;
        A[G::off(s) + c] = (c >= r) ? 0.0 : A[G::off(s) + c];
      });
    });

    // forward substitution x <- L^{-1} x for NV right-hand sides
    auto fwd = [&](auto& x) {
      constexpr int NV = std::extent<std::remove_reference_t<decltype(x)>, 0>::value;
      sfor<0, K>([&](auto c_) {
        constexpr int c = c_.value;
        constexpr int sc = c / 16;
        constexpr int lc = G::lane_of(c);
        sfor<0, NV>([&](auto v_) {
          constexpr int v = v_.value;
          const double xc = bcast<lc>(x[v][sc] * idg[sc]);
          sfor<0, NS>([&](auto s_) {
            constexpr int s = s_.value;
            if constexpr (16 * s + 15 > c)
              x[v][s] = __builtin_fma(-A[G::off(s) + c], xc, x[v][s]);
          });
        });
      });
      sfor<0, NV>([&](auto v_) {
        sfor<0, NS>([&](auto s_) { x[v_.value][s_.value] *= idg[s_.value]; });
      });
    };
    fwd(rhs);  // Liy, LiX

    // ---------------- u = L^{-T} e_last via L in LDS ----------------
    sfor<0, NS>([&](auto s_) {
      constexpr int s = s_.value;
      const int r = row_of(s, l);
      sfor<0, G::len(s)>([&](auto c_) {
        constexpr int c = c_.value;
        if (c < r && r < K) Lp[grp][r * (r + 1) / 2 + c] = A[G::off(s) + c];
      });
    });
    double uu[NS];
    sfor<0, NS>([&](auto s_) { uu[s_.value] = (row_of(s_.value, l) == K - 1) ? 1.0 : 0.0; });
    __syncthreads();
    sfor<0, K>([&](auto cc_) {
      constexpr int r = K - 1 - cc_.value;
      constexpr int sr = r / 16;
      constexpr int lr = G::lane_of(r);
      const double ur = bcast<lr>(uu[sr] * idg[sr]);
      sfor<0, NS>([&](auto s_) {
        constexpr int s = s_.value;
        if constexpr (16 * s < r) {
          const int row = row_of(s, l);
          if constexpr (16 * s + 15 < r) {
            uu[s] = __builtin_fma(-Lp[grp][r * (r + 1) / 2 + row], ur, uu[s]);
          } else {
            const double lv = Lp[grp][r * (r + 1) / 2 + (row < r ? row : r)];
            uu[s] = (row < r) ? __builtin_fma(-lv, ur, uu[s]) : uu[s];
          }
        }
      });
    });
    sfor<0, NS>([&](auto s_) {
      constexpr int s = s_.value;
      uu[s] *= idg[s];
      const int r = row_of(s, l);
      if (r < K) {
        uv[grp][r] = uu[s];
#pragma unroll
        for (int g = 0; g < NG; ++g) gv[grp][g][r] = 0.0;
      }
    });
    __syncthreads();

    // ---------------- phase 2: g_rho = dSigma/drho * u (tournament) ----------------
    {
      constexpr int KO = (K & 1) ? K : K + 1;
      constexpr int M2 = (KO - 1) / 2;
      constexpr int NSUB = (M2 + 15) / 16;
      for (int t = 0; t < KO; ++t) {
        sfor<0, NSUB>([&](auto j_) {
          const int sidx = 1 + l + 16 * j_.value;
          int a = t + sidx;
          a -= (a >= KO) ? KO : 0;
          int b = t - sidx;
          b += (b < 0) ? KO : 0;
          const bool ra = (a < q) || (a == K - 1);
          const bool rb = (b < q) || (b == K - 1);
          if (sidx <= M2 && ra && rb) {
            double h2 = 0.0, h2g1 = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const double dz = zs[grp][a][k] - zs[grp][b][k];
              const double dz2 = dz * dz;
              h2 += dz2;
              h2g1 = __builtin_fma(cf.msk[k], dz2, h2g1);
            }
            double h, hinv;
            dist_from_sq(h2, h, hinv);
            const double E = exp(-h);
            const double sF =
                cf.sigma2 * E * __builtin_fma(cf.a1, h, __builtin_fma(cf.a2, hinv, cf.a0));
            const double ua = uv[grp][a], ub = uv[grp][b];
            const double D0 = sF * ((NG == 2) ? (h2 - h2g1) : h2) * cf.ir[0];
            atomicAdd(&gv[grp][0][a], D0 * ub);
            atomicAdd(&gv[grp][0][b], D0 * ua);
            if constexpr (NG == 2) {
              const double D1 = sF * h2g1 * cf.ir[1];
              atomicAdd(&gv[grp][1][a], D1 * ub);
              atomicAdd(&gv[grp][1][b], D1 * ua);
            }
          }
        });
      }
    }
    __syncthreads();

    // ---------------- w = L^{-1} (dSigma_j u) ----------------
    double w[NR][NS];
    sfor<0, NS>([&](auto s_) {
      constexpr int s = s_.value;
      const int r = row_of(s, l);
      const int rc = r < K ? r : K - 1;
#pragma unroll
      for (int g = 0; g < NG; ++g) w[g][s] = (r < K) ? gv[grp][g][rc] : 0.0;
      w[NG][s] = uu[s];
    });
    fwd(w);
    sfor<0, NS>([&](auto s_) { w[NG][s_.value] *= cf.sigma2; });

    // ---------------- per-neighbourhood sums ----------------
    double part[NPART];
    sfor<0, NPART>([&](auto e_) { part[e_.value] = 0.0; });
    sfor<0, NS>([&](auto s_) {
      constexpr int s = s_.value;
      const double keep = (row_of(s, l) < K - 1) ? 1.0 : 0.0;
      sfor<0, NR>([&](auto j_) {
        part[j_.value] = __builtin_fma(keep * w[j_.value][s], rhs[0][s], part[j_.value]);
      });
      sfor<0, NR>([&](auto j_) {
        sfor<0, PC>([&](auto t_) {
          constexpr int e = NR + j_.value * PC + t_.value;
          part[e] = __builtin_fma(keep * w[j_.value][s], rhs[1 + t_.value][s], part[e]);
        });
      });
      sfor<0, NR>([&](auto j_) {
        constexpr int j = j_.value;
        sfor<j, NR>([&](auto k_) {
          constexpr int k = k_.value;
          constexpr int e = NR + NR * PC + (j * (2 * NR - j + 1)) / 2 + (k - j);
          part[e] = __builtin_fma(keep * w[j][s], w[k][s], part[e]);
        });
      });
    });
    sfor<0, NPART>([&](auto e_) { part[e_.value] = row_allreduce(part[e_.value]); });

    if (active && l == LS) {
      const double Lyq = rhs[0][SS];
      bool nonfinite = !(__builtin_isfinite(Lyq));
      sfor<0, PC>([&](auto t_) { nonfinite |= !(__builtin_isfinite(rhs[1 + t_.value][SS])); });
      // parameter j: 0 -> sigma2 (w = e_last / sigma2), j >= 1 -> w[j - 1]
      auto wq = [&](auto j_) -> double {
        constexpr int j = decltype(j_)::value;
        if constexpr (j == 0) return inv_sigma2; else return w[j - 1][SS];
      };
      auto Sy = [&](auto j_) -> double {
        constexpr int j = decltype(j_)::value;
        if constexpr (j == 0) return 0.0; else return part[j - 1];
      };
      auto SX = [&](auto j_, auto t_) -> double {
        constexpr int j = decltype(j_)::value, t = decltype(t_)::value;
        if constexpr (j == 0) return 0.0; else return part[NR + (j - 1) * PC + t];
      };
      auto Gjk = [&](auto j_, auto k_) -> double {
        constexpr int j = decltype(j_)::value, k = decltype(k_)::value;
        if constexpr (j == 0 || k == 0) {
          return 0.0;
        } else {
          constexpr int a = (j < k ? j : k) - 1, b = (j < k ? k : j) - 1;
          return part[NR + NR * PC + (a * (2 * NR - a + 1)) / 2 + (b - a)];
        }
      };
      auto LXq = [&](auto t_) -> double { return rhs[1 + decltype(t_)::value][SS]; };
      double* ac = acc[grp];
      ac[0] += log(vself);
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
    if (active && badnn) {
      atomicOr(&status[0], 2);
      atomicMin(&status[1], (int32_t)i);
    }
    __syncthreads();
  }
  __syncthreads();
  for (int e = threadIdx.x; e < NRAW; e += kThreads)
    partials[(size_t)blockIdx.x * NRAW + e] = ((acc[0][e] + acc[1][e]) + acc[2][e]) + acc[3][e];
}

// Host-side launcher of one instantiation.
template <int K, int PC, int NG>
hipError_t launch_sums(int grid, hipStream_t stream, int m, int d, int nspace, int nu,
                       const double* locs, const int32_t* NN, const double* y, const double* X,
                       const double* covparms, int64_t i0, int64_t i1, double* partials,
                       int32_t* status) {
  hipLaunchKernelGGL((sums_kernel<K, PC, NG>), dim3(grid), dim3(kThreads), 0, stream, m, d,
                     nspace, nu, locs, NN, y, X, covparms, i0, i1, partials, status);
  return hipGetLastError();
}

using launch_fn = hipError_t (*)(int, hipStream_t, int, int, int, int, const double*,
                                 const int32_t*, const double*, const double*, const double*,
                                 int64_t, int64_t, double*, int32_t*);

// Instantiated K values (K >= m + 1 is padded with identity rows).
constexpr int kNumK = 3;
constexpr int kKs[kNumK] = {11, 21, 31};

}  // namespace vecchia

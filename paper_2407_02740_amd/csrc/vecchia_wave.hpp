// Launch interface of the per-neighbourhood kernel for covariances with one
// range per coordinate (many covariance parameters), used by the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace vecchia_aniso {

constexpr int kMaxD = 32;  // coordinates, each with its own range
constexpr int kMaxK = 64;  // neighbourhood size m + 1
constexpr int kMaxPc = 3;  // covariates

struct AnisoArgs {
  int m, d, p, nu;  // nu: 0 -> 1/2, 1 -> 3/2, 2 -> 5/2
  const double* locs;
  const int32_t* NN;
  const double* y;
  const double* X;
  const double* covparms;  // (sigma2, rho_1..rho_d, tau2), read on the device
  int64_t i0, i1;
  double* partials;  // [grid][nraw]
  int32_t* status;
};

// Workgroups (one wave, one neighbourhood at a time each) for `total`
// observations on the current device.
int aniso_grid(int64_t total);

// Launch over [i0, i1) with `grid` workgroups; partial sums per workgroup.
hipError_t launch_aniso(const AnisoArgs& a, int grid, hipStream_t st);

}  // namespace vecchia_aniso

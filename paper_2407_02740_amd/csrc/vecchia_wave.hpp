// Launch interface of the wave-per-neighbourhood kernel (many covariance
// parameters, or neighbourhoods beyond the fused kernel's sizes), used by
// the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace vecchia_wave {

constexpr int kMaxD = 32;  // coordinates, each with its own range
constexpr int kMaxK = 64;  // neighbourhood size m + 1
constexpr int kMaxPc = 3;  // covariates
constexpr int kMaxBlock = 8;  // observations per block (grouped Vecchia, d <= 4)

struct WaveArgs {
  int m, d, p, nu;  // nu: 0 -> 1/2, 1 -> 3/2, 2 -> 5/2
  // range parameters: R = 1 (isotropic), 2 (space-time: coordinates
  // < nspace use the first), or d (one per coordinate)
  int family, nspace, R;
  const double* locs;
  const int32_t* NN;
  const double* y;
  const double* X;
  const double* covparms;  // (sigma2, rho_1..rho_R, tau2), read on the device
  int64_t i0, i1;    // observations, or blocks when block_start is set
  // grouped: blocks [block_start[b], block_start[b + 1]) of at most gmax
  // observations, conditioning sets cond[cond_start[b] .. cond_start[b + 1])
  // of at most m earlier observations; n bounds the block ends
  const int64_t* block_start;
  const int64_t* cond_start;
  const int32_t* cond;
  int64_t ncond;  // entries of cond
  int gmax;
  int64_t n;
  double* partials;  // [grid][nraw]
  int32_t* status;
};

// Workgroups (one wave, one neighbourhood at a time each) for `total`
// observations on the current device.
int wave_grid(int64_t total);

// Launch over [i0, i1) with `grid` workgroups; partial sums per workgroup.
hipError_t launch_wave(const WaveArgs& a, int grid, hipStream_t st);

}  // namespace vecchia_wave

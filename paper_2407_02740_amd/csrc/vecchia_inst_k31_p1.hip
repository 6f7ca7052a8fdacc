// Instantiations of the fused per-neighbourhood kernel for K = 31
// (m <= 30) and p = 1 covariates, isotropic and space-time ranges.
#include "vecchia_kernels.hpp"

namespace vecchia {
template hipError_t launch_sums<31, 1, 1>(int, hipStream_t, int, int, int, int, const double*,
                                          const int32_t*, const double*, const double*,
                                          const double*, int64_t, int64_t, double*, int32_t*);
template hipError_t launch_sums<31, 1, 2>(int, hipStream_t, int, int, int, int, const double*,
                                          const int32_t*, const double*, const double*,
                                          const double*, int64_t, int64_t, double*, int32_t*);
}  // namespace vecchia

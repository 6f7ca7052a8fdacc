// Instantiations of the fused per-neighbourhood kernel for K = 21
// (m <= 20) and p = 3 covariates, isotropic and space-time ranges.
#include "vecchia_kernels.hpp"

namespace vecchia {
template hipError_t launch_sums<21, 3, 1>(int, hipStream_t, int, int, int, int, const double*,
                                          const int32_t*, const double*, const double*,
                                          const double*, int64_t, int64_t, double*, int32_t*);
template hipError_t launch_sums<21, 3, 2>(int, hipStream_t, int, int, int, int, const double*,
                                          const int32_t*, const double*, const double*,
                                          const double*, int64_t, int64_t, double*, int32_t*);
}  // namespace vecchia

// Instantiations of the fused per-neighbourhood kernel for K = 11
// (m <= 10) and p = 1 covariate: isotropic and space-time ranges, each in
// the sums, adjoint and loglik-only modes.
#include "vecchia_kernels.hpp"

namespace vecchia {
#define VECCHIA_INSTANTIATE(K, PC, NG, MODE) template VECCHIA_LAUNCH_SIG(K, PC, NG, MODE)
VECCHIA_FOR_MODES(VECCHIA_INSTANTIATE, 11, 1);
}  // namespace vecchia

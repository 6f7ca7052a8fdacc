// Instantiations of the fused per-neighbourhood kernel for K = 35
// (31 <= m <= 34), p = 2 covariates and isotropic range: the
// single-problem modes (sums, adjoint, loglik-only, weights); this size has
// no batched class.
#include "vecchia_kernels.hpp"

namespace vecchia {
#define VECCHIA_INSTANTIATE(K, PC, NG, MODE, B) template VECCHIA_LAUNCH_SIG(K, PC, NG, MODE, B)
VECCHIA_FOR_NG_SINGLE(VECCHIA_INSTANTIATE, 35, 2, 1);
}  // namespace vecchia

// Instantiations of the fused per-neighbourhood kernel for K = 35
// (31 <= m <= 34), p = 3 covariates and space-time ranges: the
// single-problem modes (sums, adjoint, loglik-only, weights); this size has
// no batched class.
#include "vecchia_kernels.hpp"

namespace vecchia {
#define VECCHIA_INSTANTIATE(K, PC, NG, MODE, B) template VECCHIA_LAUNCH_SIG(K, PC, NG, MODE, B)
VECCHIA_FOR_NG_SINGLE(VECCHIA_INSTANTIATE, 35, 3, 2);
}  // namespace vecchia

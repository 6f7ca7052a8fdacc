// Instantiations of the fused per-neighbourhood kernel for K = 21
// (m <= 20), p = 3 covariates and isotropic range: the sums, adjoint and
// loglik-only modes of the single-problem kernel and the batched sums kernel.
#include "vecchia_kernels.hpp"

namespace vecchia {
#define VECCHIA_INSTANTIATE(K, PC, NG, MODE, B) \
  template VECCHIA_LAUNCH_SIG(K, PC, NG, MODE, B); \
  template VECCHIA_RESIDENT_SIG(K, PC, NG, MODE, B)
VECCHIA_FOR_NG(VECCHIA_INSTANTIATE, 21, 3, 1);
}  // namespace vecchia

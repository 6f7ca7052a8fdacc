"""Vecchia oracle: plain FP64 CPU reference implementation.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call this package.  The GPU
library never links or calls it, and it shares no code with the GPU library.

Parity status of each function (what pins it, see ``tests/test_oracle_pins.py``):
  raw_sums      pinned: dense exact GP at full conditioning (Section 2.1, A5),
                joint-minus-marginal dense forms at any m, AR(1) closed form
                for the 1-D exponential, m = 0 closed form, sigma2 identities,
                finite differences of the log-likelihood; anisotropic sums
                collapse to the isotropic ones at equal ranges and transform
                as they must under coordinate permutation and stretching.
  cov_matrix    pinned: Matern via the Bessel-K definition (scipy), and
                finite differences for the parameter derivatives; the
                anisotropic family (a range per coordinate) equals the
                unit-range isotropic one on rescaled coordinates, and the
                isotropic one when the ranges are equal.
  combine       pinned through the dense exact GP and the AR(1) closed form.
  at_beta       pinned: central finite differences in theta at a fixed beta
                away from beta_hat, the dense reverse-mode expression of the
                gradient, and agreement with combine at beta_hat.
  kriging_predict pinned: with every observation as a neighbour it equals the
                dense Gaussian-process conditional; at an observed location
                without nugget it interpolates (mean = y, variance = 0).
  kriging_weights pinned: the loglik sums rebuilt from its weights and
                variances equal raw_sums' (a different code path, C, Neumaier
                sums); b = 0 and v = 1 + tau2 when the neighbours are far.
  grouped_raw_sums  (grouped.py) pinned: blocks of one observation equal
                raw_sums (the C code, a different implementation); one block
                of everything, and two blocks with full conditioning, equal the
                dense exact GP; every block equals the joint-minus-marginal
                dense expression; finite differences of the log-likelihood.
  fisher_step   pinned: the Eq. (4) update is a fixed point at the MLE of the
                AR(1) closed form (scipy optimiser).
"""

from .oracle import (  # noqa: F401
    FAMILY_ANISO,
    FAMILY_ISO,
    FAMILY_SPACETIME,
    OracleError,
    at_beta,
    build,
    combine,
    cov_matrix,
    fisher_step,
    fit,
    kriging_predict,
    kriging_weights,
    loglik_grad_info,
    nparms,
    nraw,
    raw_sums,
    unpack_raw,
)
from .grouped import grouped_raw_sums  # noqa: E402,F401

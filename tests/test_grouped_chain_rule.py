"""The identity that lets grouped Vecchia (Section 2.1) run on the
single-observation kernel, checked on the oracle: a block's conditional
density p(y_B | y_N) is the product of its members' one-observation
conditionals, member k conditioned on N and on members 0..k-1 (the chain rule
of the Gaussian density), and the expected information of the block
conditional is the sum of the factors' (a factor's score has mean zero given
everything the later factors condition on).  So every raw sum of a grouping
-- the loglik terms, their derivatives and the information -- equals that of
blocks of one whose conditioning sets are N plus the earlier members.

The block side is the oracle's multivariate formula (W, V, joint-minus-
marginal sums); the sequential side is its blocks-of-one path, itself pinned
to the single-observation C oracle: the two share no algebra."""

import numpy as np
import pytest

import oracle
from paper_2407_02740_amd import synthetic as S

ISO, ST, AN = oracle.FAMILY_ISO, oracle.FAMILY_SPACETIME, oracle.FAMILY_ANISO


def _sequential(bs, cs, cond):
    """Blocks of one: observation i of block b conditioned on N_b and the
    members of b before it."""
    rows = []
    for b in range(len(bs) - 1):
        nb = list(cond[cs[b]:cs[b + 1]])
        for i in range(bs[b], bs[b + 1]):
            rows.append(nb + list(range(bs[b], i)))
    sbs = np.arange(bs[0], bs[-1] + 1)
    scs = np.r_[0, np.cumsum([len(r) for r in rows])]
    scond = np.array([j for r in rows for j in r], dtype=np.int32)
    return sbs, scs, scond


def _problem(n, d, g, m, family, seed, p):
    rng = np.random.default_rng(seed)
    locs = rng.random((n, d))
    order, bs, cs, cond = S.group_cells(locs, g, m, seed=seed)
    locs = locs[order]
    y = rng.standard_normal(n) + 0.4 * np.sin(5 * locs[:, 0])
    X = np.column_stack([np.ones(n)] + [rng.standard_normal(n) for _ in range(p - 1)])
    cp = {ISO: np.array((1.3, 0.12, 0.05)), ST: np.array((1.1, 0.2, 0.4, 0.08)),
          AN: np.concatenate([[1.2], np.linspace(0.1, 0.3, d), [0.06]])}[family]
    return locs, y, X, cp, bs, cs, cond


@pytest.mark.parametrize("family,nu,d,g,m,p", [(ISO, 0.5, 2, 2, 8, 1), (ISO, 1.5, 2, 4, 10, 2),
                                               (ISO, 2.5, 2, 8, 6, 1), (ST, 0.5, 3, 4, 8, 1),
                                               (AN, 1.5, 3, 3, 7, 2)])
def test_block_sums_equal_sequential_single_conditionals(family, nu, d, g, m, p):
    locs, y, X, cp, bs, cs, cond = _problem(360, d, g, m, family, seed=41 + g, p=p)
    assert np.max(np.diff(bs)) > 1  # real blocks
    got = oracle.grouped_raw_sums(locs, y, X, cp, bs, cs, cond, family, nu, nspace=2)
    sbs, scs, scond = _sequential(bs, cs, cond)
    ref = oracle.grouped_raw_sums(locs, y, X, cp, sbs, scs, scond, family, nu, nspace=2)
    np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_a_sub_range_of_blocks():
    """The sums of a run of blocks that does not start at observation 0."""
    locs, y, X, cp, bs, cs, cond = _problem(300, 2, 4, 9, ISO, seed=47, p=1)
    b0, b1 = 20, 55
    sbs = bs[b0:b1 + 1]
    scs = cs[b0:b1 + 1] - cs[b0]
    scond = cond[cs[b0]:cs[b1]]
    got = oracle.grouped_raw_sums(locs, y, X, cp, sbs, scs, scond, ISO, 1.5)
    qbs, qcs, qcond = _sequential(sbs, scs, scond)
    ref = oracle.grouped_raw_sums(locs, y, X, cp, qbs, qcs, qcond, ISO, 1.5)
    np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())

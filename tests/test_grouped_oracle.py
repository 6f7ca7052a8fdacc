"""Pins of the grouped Vecchia oracle (block conditionals, oracle/grouped.py)
by routes that share none of its algebra: the single-observation C oracle,
the dense exact Gaussian-process likelihood, the joint-minus-marginal dense
expression of every sum, and finite differences."""

import numpy as np
import pytest

import oracle
from paper_2407_02740_amd import synthetic as S
from test_oracle_pins import _dense_exact, _full_nn, _joint_minus_marginal, _problem

ISO, ST, AN = oracle.FAMILY_ISO, oracle.FAMILY_SPACETIME, oracle.FAMILY_ANISO


def _singletons(NN):
    n, m1 = NN.shape
    rows = [NN[i, 1:1 + min(i, m1 - 1)] for i in range(n)]
    cs = np.r_[0, np.cumsum([len(r) for r in rows])]
    return np.arange(n + 1), cs, np.concatenate(rows).astype(np.int32)


@pytest.mark.parametrize("family,nu,p,d", [(ISO, 0.5, 1, 2), (ISO, 2.5, 2, 2), (ST, 1.5, 1, 3),
                                           (AN, 0.5, 3, 3)])
def test_blocks_of_one_are_the_single_observation_sums(family, nu, p, d):
    locs, NN, y, X, cp = _problem(300, 9, d=d, p=p, family=family, nu=nu, seed=31)
    bs, cs, cond = _singletons(NN)
    got = oracle.grouped_raw_sums(locs, y, X, cp, bs, cs, cond, family, nu, nspace=2)
    ref = oracle.raw_sums(locs, NN, y, X, cp, family, nu, nspace=2)
    np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


@pytest.mark.parametrize("family,nu,p", [(ISO, 0.5, 1), (ISO, 1.5, 2), (ST, 0.5, 1)])
def test_full_conditioning_is_the_exact_gp(family, nu, p):
    n = 36
    d = 2 if family == ISO else 3
    locs, _, y, X, cp = _problem(n, 5, d=d, p=p, family=family, nu=nu, seed=32)
    ll, grad, info, beta = _dense_exact(locs, y, X, cp, family, nu, nspace=2)
    P = len(cp)
    for bs, cs, cond in [
        (np.array([0, n]), np.array([0, 0]), np.zeros(0, np.int32)),                      # one block
        (np.array([0, 15, n]), np.array([0, 0, 15]), np.arange(15, dtype=np.int32)),       # two
        (np.array([0, 1, 7, 20, n]), np.array([0, 0, 1, 8, 28]),                           # four
         np.concatenate([[0], np.arange(7), np.arange(20)]).astype(np.int32)),
    ]:
        raw = oracle.grouped_raw_sums(locs, y, X, cp, bs, cs, cond, family, nu, nspace=2)
        res = oracle.combine(raw, n, p, P)
        assert abs(res["loglik"] - ll) <= 1e-11 * abs(ll)
        sd = np.sqrt(np.diag(info))
        assert np.all(np.abs(res["grad"] - grad) <= 1e-9 * np.maximum(np.abs(grad), sd))
        np.testing.assert_allclose(res["info"], info, rtol=1e-10)
        np.testing.assert_allclose(res["betahat"], beta, rtol=1e-9, atol=1e-11)


def _block_joint_minus_marginal(locs, y, X, cp, bs, cs, cond, family, nu):
    """Every sum as (dense expression over N u B) - (over N), block by block,
    through the single-observation helper on a two-row 'NNarray' per block."""
    P, p = len(cp), X.shape[1]
    tot = None
    for b in range(len(bs) - 1):
        N = list(cond[cs[b]:cs[b + 1]])
        B = list(range(bs[b], bs[b + 1]))
        idx = N + B
        # local problem: the joint set in local order; the last |B| rows are
        # the block, each conditioning on everything before it in the block
        # order (N first), which chains to the joint minus the marginal of N
        k = len(idx)
        NNl = np.full((k, k), -1, dtype=np.int32)
        for i in range(k):
            NNl[i, 0] = i
            NNl[i, 1:i + 1] = np.arange(i)
        r = _joint_minus_marginal(locs[idx], NNl, y[idx], X[idx], cp, family, nu, nspace=2)
        # keep only the block rows' terms: joint over all k minus the first |N|
        if len(N):
            r0 = _joint_minus_marginal(locs[N], NNl[:len(N), :len(N)], y[N], X[N], cp, family,
                                       nu, nspace=2)
            r = {key: np.asarray(r[key]) - np.asarray(r0[key]) for key in r}
        tot = r if tot is None else {key: tot[key] + np.asarray(r[key]) for key in tot}
    return tot


def test_every_sum_is_joint_minus_marginal():
    locs, NN, y, X, cp = _problem(400, 6, d=2, p=2, family=ISO, nu=1.5, seed=33)
    order, bs, cs, cond = S.group_cells(locs, 3, 6, seed=3)
    locs, y, X = locs[order], y[order], X[order]
    raw = oracle.grouped_raw_sums(locs, y, X, cp, bs, cs, cond, ISO, 1.5)
    got = oracle.unpack_raw(raw, 2, 3)
    ref = _block_joint_minus_marginal(locs, y, X, cp, bs, cs, cond, ISO, 1.5)
    for key in got:
        a, b = np.asarray(got[key]), np.asarray(ref[key])
        np.testing.assert_allclose(a, b, rtol=1e-8, atol=1e-8 * (1 + np.abs(b).max()), err_msg=key)


def test_gradient_matches_finite_differences():
    locs, NN, y, X, cp = _problem(600, 8, d=3, p=1, family=ST, nu=0.5, seed=34)
    order, bs, cs, cond = S.group_cells(locs, 4, 8, seed=4)
    locs, y, X = locs[order], y[order], X[order]

    def ll(th):
        raw = oracle.grouped_raw_sums(locs, y, X, th, bs, cs, cond, ST, 0.5, nspace=2)
        return oracle.combine(raw, len(y), 1, 4)

    res = ll(cp)
    sd = np.sqrt(np.diag(res["info"]))
    assert np.all(np.linalg.eigvalsh(res["info"]) > 0)
    np.testing.assert_allclose(res["info"], res["info"].T, rtol=1e-12)
    for j in range(4):
        h = 1e-5 * cp[j]
        a, b = cp.copy(), cp.copy()
        a[j] += h
        b[j] -= h
        fd = (ll(a)["loglik"] - ll(b)["loglik"]) / (2 * h)
        assert abs(fd - res["grad"][j]) <= 1e-6 * max(abs(fd), sd[j]), (j, fd, res["grad"][j])


def test_malformed_blocks_are_reported():
    locs, NN, y, X, cp = _problem(50, 4, seed=35)
    with pytest.raises(oracle.OracleError):
        oracle.grouped_raw_sums(locs, y, X, cp, [0, 10, 50], [0, 0, 3], [2, 11, 3], ISO, 0.5)

"""Grouped Vecchia sums: plain FP64 reference.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Grouping (Section 2.1: conditioning on the joint distribution of several
observations at once, which cuts the number of likelihood terms and sharpens
the approximation) replaces the conditional density of one observation by
that of a block.  The ordered observations are split into consecutive
blocks B_1, B_2, ...; block b has a conditioning set N_b of earlier
observations (indices below the block's first member), and the likelihood
is the product of the block conditionals p(y_B | y_N).

Written from the definition of a Gaussian conditional: with Sigma over
J = (N, B), the weights W = Sigma_NN^-1 Sigma_NB, the conditional covariance
V = Sigma_BB - Sigma_NB' W, residuals e_y = y_B - W' y_N and
e_X = X_B - W' X_N, each block adds
    logdet += log det V,        ySy += e_y' V^-1 e_y,
    XSX    += e_X' V^-1 e_X,    ySX += e_X' V^-1 e_y,
and for each covariance parameter theta_j, with
    dW_j = Sigma_NN^-1 (dSigma_NB - dSigma_NN W),
    dV_j = dSigma_BB - dSigma_NB' W - W' dSigma_NB + W' dSigma_NN W,
    de_y = -dW_j' y_N,  de_X = -dW_j' X_N:
    dlogdet_j += tr(V^-1 dV_j)
    dySy_j    += 2 de_y' V^-1 e_y - e_y' V^-1 dV_j V^-1 e_y
    dXSX_j    += de_X' V^-1 e_X + e_X' V^-1 de_X - e_X' V^-1 dV_j V^-1 e_X
    dySX_j    += de_X' V^-1 e_y + e_X' V^-1 de_y - e_X' V^-1 dV_j V^-1 e_y
    ainfo_jk  += tr(V^-1 dV_j V^-1 dV_k) / 2 + tr(V^-1 dW_j' Sigma_NN dW_k)
(the expected information of the block conditional with y_N drawn from its
marginal).  A block of one observation with N its neighbour row is the
single-observation form of vecchia_oracle.c.  Raw-sum layout as there.
"""

from __future__ import annotations

import numpy as np

from .oracle import OracleError, cov_matrix, nparms, nraw, unpack_raw  # noqa: F401


def grouped_raw_sums(locs, y, X, covparms, block_start, cond_start, cond, family=0, nu=0.5,
                     nspace=0):
    """Sums over the blocks [block_start[b], block_start[b + 1]) with
    conditioning sets cond[cond_start[b]:cond_start[b + 1]]."""
    locs = np.asarray(locs, dtype=np.float64)
    if locs.ndim == 1:
        locs = locs[:, None]
    y = np.asarray(y, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    n, d = locs.shape
    p = X.shape[1]
    cp = np.asarray(covparms, dtype=np.float64)
    P = nparms(family, d)
    bs = np.asarray(block_start, dtype=np.int64)
    cs = np.asarray(cond_start, dtype=np.int64)
    cond = np.asarray(cond, dtype=np.int64)
    nb = len(bs) - 1
    logdet = ySy = 0.0
    XSX, ySX = np.zeros((p, p)), np.zeros(p)
    dlogdet, dySy = np.zeros(P), np.zeros(P)
    dXSX, dySX = np.zeros((P, p, p)), np.zeros((P, p))
    ainfo = np.zeros((P, P))
    for b in range(nb):
        B = np.arange(bs[b], bs[b + 1])
        N = cond[cs[b]:cs[b + 1]]
        if len(B) == 0 or np.any(N < 0) or np.any(N >= bs[b]):
            raise OracleError(-3, int(bs[b]))
        c = len(N)
        J = np.concatenate([N, B])
        S, dS = cov_matrix(locs[J], cp, family, nu, nspace)
        SNN, SNB, SBB = S[:c, :c], S[:c, c:], S[c:, c:]
        W = np.linalg.solve(SNN, SNB) if c else np.zeros((0, len(B)))
        V = SBB - SNB.T @ W
        try:
            np.linalg.cholesky(V)
        except np.linalg.LinAlgError:
            raise OracleError(-2, int(bs[b])) from None
        Vi = np.linalg.inv(V)
        ey = y[B] - W.T @ y[N]
        eX = X[B] - W.T @ X[N]
        logdet += np.linalg.slogdet(V)[1]
        ySy += ey @ Vi @ ey
        XSX += eX.T @ Vi @ eX
        ySX += eX.T @ Vi @ ey
        dW, dV = [], []
        for j in range(P):
            dNN, dNB, dBB = dS[j][:c, :c], dS[j][:c, c:], dS[j][c:, c:]
            dWj = np.linalg.solve(SNN, dNB - dNN @ W) if c else np.zeros((0, len(B)))
            dVj = dBB - dNB.T @ W - W.T @ dNB + W.T @ dNN @ W
            dey = -dWj.T @ y[N]
            deX = -dWj.T @ X[N]
            A = Vi @ dVj @ Vi
            dlogdet[j] += np.trace(Vi @ dVj)
            dySy[j] += 2.0 * dey @ Vi @ ey - ey @ A @ ey
            dXSX[j] += deX.T @ Vi @ eX + eX.T @ Vi @ deX - eX.T @ A @ eX
            dySX[j] += deX.T @ Vi @ ey + eX.T @ Vi @ dey - eX.T @ A @ ey
            dW.append(dWj)
            dV.append(dVj)
        for j in range(P):
            for k in range(P):
                ainfo[j, k] += 0.5 * np.trace(Vi @ dV[j] @ Vi @ dV[k]) + \
                    np.trace(Vi @ dW[j].T @ SNN @ dW[k])
    return np.concatenate([[logdet, ySy], XSX.ravel(), ySX, dlogdet, dySy, dXSX.ravel(),
                           dySX.ravel(), ainfo.ravel()])

"""ctypes binding of the C oracle plus the combine and Fisher-scoring steps.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every function here is
written from the paper's statement of the method:

* ``raw_sums``   -- the sums of Algorithm 1 (Section 3) over observations,
                    computed by ``vecchia_oracle.c`` in the conditional-Gaussian
                    (kriging-weight) form.
* ``combine``    -- the "separate function" of Section 3 that turns the sums
                    into the profile log-likelihood, its gradient and the Fisher
                    information, with the mean parameters profiled out
                    (generalised least squares, Section 2.1 / Section 3).
* ``at_beta``    -- the same log-likelihood and theta-gradient at a given
                    (not profiled) mean vector beta.
* ``kriging_predict`` -- conditional mean and variance at new points given
                    their observed neighbours.
* ``kriging_weights`` -- per observation the weights and log conditional
                    variance of its conditional density (Eq. 3), solved
                    densely from the definition.
* ``fisher_step``-- one Fisher-scoring update, Eq. (4), taken on the log scale
                    of the (positive) covariance parameters with a unit cap on
                    the step length.

Scale convention: the paper's Eq. (1)-(2) are twice the usual log-likelihood
and score.  Here loglik = -1/2 (n log 2 pi + logdet + quadratic form), its
gradient, and the matching information ainfo are reported; Eq. (4)'s step is
the same under either scaling.
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

FAMILY_ISO = 0
FAMILY_SPACETIME = 1
FAMILY_ANISO = 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vecchia_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()

_ERRORS = {-1: "invalid argument", -2: "covariance not positive definite", -3: "bad NNarray row"}


class OracleError(RuntimeError):
    def __init__(self, code: int, bad_i: int):
        super().__init__(f"oracle: {_ERRORS.get(code, code)} at observation {bad_i}")
        self.code = code
        self.bad_i = bad_i


def build(force: bool = False) -> str:
    """Compile the C oracle into ``oracle/liboracle.so`` (plain gcc, IEEE FP64)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-std=c11", "-shared", "-fPIC",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build()
            lib = ctypes.CDLL(_LIB)
            dp = ctypes.POINTER(ctypes.c_double)
            ip = ctypes.POINTER(ctypes.c_int32)
            lib.oracle_raw_sums.restype = ctypes.c_int
            lib.oracle_raw_sums.argtypes = [
                ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                ctypes.c_double, ctypes.c_int, dp, ip, dp, dp, dp, ctypes.c_int64,
                ctypes.c_int64, dp, ctypes.POINTER(ctypes.c_int64)]
            lib.oracle_cov_matrix.restype = ctypes.c_int
            lib.oracle_cov_matrix.argtypes = [
                ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, dp,
                dp, dp]
            lib.oracle_nparms.restype = ctypes.c_int
            lib.oracle_nparms.argtypes = [ctypes.c_int, ctypes.c_int]
            lib.oracle_nraw.restype = ctypes.c_int
            lib.oracle_nraw.argtypes = [ctypes.c_int, ctypes.c_int]
            _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def nparms(family: int, d: int | None = None) -> int:
    """Number of covariance parameters: (sigma2, rho, tau2), (sigma2,
    rho_space, rho_time, tau2), or (sigma2, rho_1..rho_d, tau2)."""
    if family == FAMILY_ANISO:
        if d is None:
            raise ValueError("the anisotropic family needs the dimension d")
        return d + 2
    return {FAMILY_ISO: 3, FAMILY_SPACETIME: 4}[family]


def nraw(p: int, P: int) -> int:
    return 2 + p * p + p + P * (2 + p * p + p) + P * P


def cov_matrix(locs, covparms, family=FAMILY_ISO, nu=0.5, nspace=0):
    """Covariance matrix of the given locations and its parameter derivatives."""
    lib = _load()
    locs = np.ascontiguousarray(locs, dtype=np.float64)
    if locs.ndim == 1:
        locs = locs[:, None]
    k, d = locs.shape
    P = nparms(family, d)
    cp = np.ascontiguousarray(covparms, dtype=np.float64)
    S = np.empty((k, k))
    dS = np.empty((P, k, k))
    st = lib.oracle_cov_matrix(k, d, _dp(locs), family, float(nu), int(nspace), _dp(cp), _dp(S),
                               _dp(dS))
    if st != 0:
        raise OracleError(st, -1)
    return S, dS


def raw_sums(locs, NN, y, X, covparms, family=FAMILY_ISO, nu=0.5, nspace=0, i0=0, i1=None,
             threads: int = 1):
    """Sums of Algorithm 1 over observations i0 <= i < i1.

    With ``threads > 1`` the observation range is split into contiguous chunks
    evaluated concurrently (the C code releases the GIL); the chunk sums are
    added with ``math.fsum``.
    """
    lib = _load()
    locs = np.ascontiguousarray(locs, dtype=np.float64)
    if locs.ndim == 1:
        locs = locs[:, None]
    n, d = locs.shape
    NN = np.ascontiguousarray(NN, dtype=np.int32)
    m = NN.shape[1] - 1
    y = np.ascontiguousarray(y, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    p = X.shape[1]
    cp = np.ascontiguousarray(covparms, dtype=np.float64)
    P = nparms(family, d)
    if cp.shape != (P,):
        raise ValueError(f"covparms must have {P} entries")
    i1 = n if i1 is None else i1
    nr = nraw(p, P)

    def run(a, b):
        raw = np.zeros(nr)
        bad = ctypes.c_int64(-1)
        st = lib.oracle_raw_sums(n, m, d, p, family, float(nu), int(nspace), _dp(locs),
                                 NN.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(y),
                                 _dp(X), _dp(cp), a, b, _dp(raw), ctypes.byref(bad))
        if st != 0:
            raise OracleError(st, bad.value)
        return raw

    if threads <= 1 or i1 - i0 < 2 * threads:
        return run(i0, i1)
    bounds = np.linspace(i0, i1, 4 * threads + 1).astype(np.int64)
    with ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(lambda ab: run(int(ab[0]), int(ab[1])), zip(bounds[:-1], bounds[1:])))
    return np.array([math.fsum(col) for col in np.stack(parts).T])


def unpack_raw(raw, p: int, P: int) -> dict:
    """Split a raw-sum vector into its named parts (documented layout)."""
    raw = np.asarray(raw, dtype=np.float64)
    o = 0

    def take(shape):
        nonlocal o
        size = int(np.prod(shape)) if shape else 1
        v = raw[o:o + size]
        o += size
        return v.reshape(shape) if shape else float(v[0])

    out = dict(logdet=take(()), ySy=take(()), XSX=take((p, p)), ySX=take((p,)),
               dlogdet=take((P,)), dySy=take((P,)), dXSX=take((P, p, p)), dySX=take((P, p)),
               ainfo=take((P, P)))
    assert o == raw.size
    return out


def combine(raw, n: int, p: int, P: int) -> dict:
    """Profile log-likelihood, gradient and Fisher information from the sums.

    beta_hat = XSX^{-1} ySX (generalised least squares at the current theta);
    loglik   = -1/2 (n log 2 pi + logdet + ySy - ySX^T beta_hat);
    grad_j   = -1/2 (dlogdet_j + dySy_j - 2 beta_hat^T dySX_j
                     + beta_hat^T dXSX_j beta_hat)   (envelope theorem);
    info     = ainfo;  betainfo = XSX.
    """
    r = unpack_raw(raw, p, P)
    beta = np.linalg.solve(r["XSX"], r["ySX"])
    loglik = -0.5 * (n * math.log(2.0 * math.pi) + r["logdet"] + r["ySy"] - r["ySX"] @ beta)
    grad = np.array([
        -0.5 * (r["dlogdet"][j] + r["dySy"][j] - 2.0 * beta @ r["dySX"][j]
                + beta @ r["dXSX"][j] @ beta) for j in range(P)])
    return dict(loglik=loglik, grad=grad, info=r["ainfo"].copy(), betahat=beta,
                betainfo=r["XSX"].copy())


def at_beta(raw, n: int, p: int, P: int, beta) -> dict:
    """Log-likelihood and its theta-gradient at a fixed mean vector beta.

    With r = y - X beta the quadratic form of Eq. (2) expands in the sums as
    ySy - 2 beta^T ySX + beta^T XSX beta, and each of its theta-derivatives
    in the derivative sums likewise:
    loglik = -1/2 (n log 2 pi + logdet + ySy - 2 beta^T ySX + beta^T XSX beta),
    grad_j = -1/2 (dlogdet_j + dySy_j - 2 beta^T dySX_j + beta^T dXSX_j beta).
    At beta = beta_hat these equal the profile values of ``combine``.
    """
    r = unpack_raw(raw, p, P)
    beta = np.asarray(beta, dtype=np.float64).reshape(p)
    quad = r["ySy"] - 2.0 * beta @ r["ySX"] + beta @ r["XSX"] @ beta
    loglik = -0.5 * (n * math.log(2.0 * math.pi) + r["logdet"] + quad)
    grad = np.array([
        -0.5 * (r["dlogdet"][j] + r["dySy"][j] - 2.0 * beta @ r["dySX"][j]
                + beta @ r["dXSX"][j] @ beta) for j in range(P)])
    return dict(loglik=loglik, grad=grad)


def kriging_weights(locs, NN, covparms, family=FAMILY_ISO, nu=0.5, nspace=0, i0=0, i1=None):
    """Per observation i in [i0, i1): the weights b = Sigma_s^-1 c of its
    q = min(i, m) neighbours (NNarray column order, zero beyond q) and
    log(v / sigma2) with v = Sigma_ii - c^T b, the conditional variance of
    Eq. (3) in correlation units.  Returns an array [i1 - i0][m + 1]."""
    NN = np.asarray(NN)
    n, m1 = NN.shape
    i1 = n if i1 is None else i1
    out = np.zeros((i1 - i0, m1))
    sigma2 = float(covparms[0])
    for i in range(i0, i1):
        q = min(i, m1 - 1)
        idx = list(NN[i, 1:q + 1]) + [i]
        S, _ = cov_matrix(np.asarray(locs)[idx], covparms, family, nu, nspace)
        c = S[:q, q]
        b = np.linalg.solve(S[:q, :q], c) if q else np.zeros(0)
        v = S[q, q] - c @ b
        out[i - i0, :q] = b
        out[i - i0, m1 - 1] = math.log(v / sigma2)
    return out


def kriging_predict(locs, y, X, locs_pred, X_pred, NN_pred, covparms, beta,
                    family=FAMILY_ISO, nu=0.5, nspace=0):
    """Conditional mean and variance of the observation process at each
    prediction point given its listed observed neighbours (the conditional
    Gaussian of Eq. 3 with the point in the self position):
      mean = x_p beta + c^T Sigma_s^-1 (y_s - X_s beta),
      var  = Sigma_pp - c^T Sigma_s^-1 c   (nugget included).
    NN_pred[j] lists observed indices (entries < 0 ignored)."""
    locs = np.asarray(locs, dtype=np.float64)
    locs_pred = np.asarray(locs_pred, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64).reshape(len(y), -1)
    X_pred = np.asarray(X_pred, dtype=np.float64).reshape(len(locs_pred), -1)
    beta = np.asarray(beta, dtype=np.float64)
    r = np.asarray(y, dtype=np.float64) - X @ beta
    mean = np.zeros(len(locs_pred))
    var = np.zeros(len(locs_pred))
    for j in range(len(locs_pred)):
        s = [int(k) for k in NN_pred[j] if k >= 0]
        pts = np.vstack([locs[s], locs_pred[j][None, :]]) if s else locs_pred[j][None, :]
        S, _ = cov_matrix(pts, covparms, family, nu, nspace)
        q = len(s)
        c = S[:q, q]
        b = np.linalg.solve(S[:q, :q], c) if q else np.zeros(0)
        mean[j] = X_pred[j] @ beta + (b @ r[s] if q else 0.0)
        var[j] = S[q, q] - c @ b
    return mean, var


def loglik_grad_info(locs, NN, y, X, covparms, family=FAMILY_ISO, nu=0.5, nspace=0,
                     threads: int = 1) -> dict:
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    raw = raw_sums(locs, NN, y, X, covparms, family, nu, nspace, threads=threads)
    d = 1 if np.ndim(locs) == 1 else np.shape(locs)[1]
    return combine(raw, len(y), X.shape[1], nparms(family, d))


def fisher_step(covparms, grad, info, max_step: float = 1.0):
    """One Fisher-scoring update, Eq. (4), on phi = log(theta).

    g_phi = theta * grad,  I_phi = diag(theta) I diag(theta),
    step = I_phi^{-1} g_phi, scaled down to length max_step if longer,
    theta_new = theta * exp(step).
    """
    th = np.asarray(covparms, dtype=np.float64)
    g = th * np.asarray(grad, dtype=np.float64)
    I = np.asarray(info, dtype=np.float64) * np.outer(th, th)
    step = np.linalg.solve(I, g)
    norm = float(np.sqrt(step @ step))
    if norm > max_step:
        step = step * (max_step / norm)
    return th * np.exp(step)


def fit(locs, NN, y, X, covparms, family=FAMILY_ISO, nu=0.5, nspace=0, iters: int = 20,
        threads: int = 1):
    """Fixed number of Fisher-scoring iterations; returns the final theta and history."""
    th = np.asarray(covparms, dtype=np.float64).copy()
    hist = []
    for _ in range(iters):
        res = loglik_grad_info(locs, NN, y, X, th, family, nu, nspace, threads=threads)
        hist.append(dict(theta=th.copy(), **res))
        th = fisher_step(th, res["grad"], res["info"])
    return th, hist

"""Neighbourhoods of 32 to 61 observations on the fused kernel's larger sizes
(K = 35 for 31 <= m <= 34, K = 41, K = 61 for 41 <= m <= 60: the paper's
m = 60 setting of its size study and its 60-neighbour kriging), in every
single-problem mode, against the CPU oracle.

Tolerances as for the smaller sizes:
  loglik   |d| <= 1e-10 |loglik|
  grad_j   |d| <= 1e-8 max(|grad_j|, sqrt(I_jj))
  I_jk     |d| <= 1e-8 max(|I_jk|, sqrt(I_jj I_kk))
  weights  |d| <= 1e-9 (b), 1e-10 (log v); predictions 1e-10 relative.
"""

import numpy as np
import pytest

import oracle
from paper_2407_02740_amd import synthetic as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from paper_2407_02740_amd import vecchia as V  # noqa: E402


def _say(msg):
    print(msg, flush=True)


def _problem(n, m, family, nu, p, seed):
    rng = np.random.default_rng(seed)
    d = 2 if family == V.FAMILY_ISO else 3
    locs = rng.random((n, d))
    locs = locs[S.maxmin_exact(locs)] if n <= 5000 else locs[S.maxmin_approx(locs, seed)]
    NN = S.find_ordered_nn(locs, m)
    y = rng.standard_normal(n) + 0.3 * np.sin(7 * locs[:, 0])
    X = np.column_stack([np.ones(n)] + [rng.standard_normal(n) for _ in range(p - 1)])
    cp = np.array((1.3, 0.15, 0.05)) if family == V.FAMILY_ISO else np.array((1.1, 0.3, 0.5, 0.1))
    return dict(locs=locs, NN=NN, y=y, X=X, covparms=cp, family=family, nu=nu,
                nspace=(2 if family == V.FAMILY_SPACETIME else 0), n=n, m=m, p=p)


def _ev(w):
    return V.Vecchia(w["locs"], w["NN"], w["y"], w["X"], w["family"], w["nu"], w["nspace"])


def _oracle(w):
    raw = oracle.raw_sums(w["locs"], w["NN"], w["y"], w["X"], w["covparms"], w["family"], w["nu"],
                          w["nspace"], threads=8)
    return raw, oracle.combine(raw, w["n"], w["p"], oracle.nparms(w["family"]))


def _check(got, ref, tag):
    assert abs(got["loglik"] - ref["loglik"]) <= 1e-10 * abs(ref["loglik"]), tag
    sd = np.sqrt(np.abs(np.diag(ref["info"])))
    assert np.all(np.abs(got["grad"] - ref["grad"])
                  <= 1e-8 * np.maximum(np.abs(ref["grad"]), sd)), (tag, got["grad"], ref["grad"])
    assert np.all(np.abs(got["info"] - ref["info"])
                  <= 1e-8 * np.maximum(np.abs(ref["info"]), np.outer(sd, sd))), tag


CASES = [(31, V.FAMILY_ISO, 0.5, 2), (34, V.FAMILY_SPACETIME, 1.5, 1), (41, V.FAMILY_ISO, 0.5, 1),
         (45, V.FAMILY_ISO, 1.5, 3), (52, V.FAMILY_SPACETIME, 2.5, 2), (60, V.FAMILY_ISO, 1.5, 1),
         (60, V.FAMILY_SPACETIME, 0.5, 3)]


@pytest.mark.parametrize("m,family,nu,p", CASES)
def test_sums_match_oracle(m, family, nu, p):
    w = _problem(900, m, family, nu, p, seed=500 + m)
    _say(f"sums m={m} fam={family} nu={nu} p={p}")
    raw, ref = _oracle(w)
    ev = _ev(w)
    got = V.unpack_out(ev.loglik_grad_info(w["covparms"]), p, ev.P)
    got_raw = ev.raw.cpu().numpy()
    r, g = oracle.unpack_raw(raw, p, ev.P), oracle.unpack_raw(got_raw, p, ev.P)
    for key in r:
        a, b = np.asarray(g[key]), np.asarray(r[key])
        assert np.max(np.abs(a - b)) <= 1e-9 * max(np.max(np.abs(b)), 1e-300), (key, a, b)
    _check(got, ref, f"m={m}")


@pytest.mark.parametrize("m,family,nu,p", CASES)
def test_loglik_and_adjoint_match_oracle(m, family, nu, p):
    w = _problem(700, m, family, nu, p, seed=600 + m)
    _say(f"loglik/adjoint m={m} fam={family} nu={nu} p={p}")
    raw, ref = _oracle(w)
    ev = _ev(w)
    out = ev.loglik(w["covparms"]).cpu().numpy()
    assert abs(out[0] - ref["loglik"]) <= 1e-10 * abs(ref["loglik"])
    bscale = np.abs(ref["betahat"]) + 1.0 / np.sqrt(np.diag(ref["betainfo"]))
    assert np.all(np.abs(out[1:1 + p] - ref["betahat"]) <= 1e-8 * bscale)
    sd = np.sqrt(np.abs(np.diag(ref["info"])))
    for beta in (ref["betahat"], ref["betahat"] + 0.4 - 0.3 * np.arange(p)):
        at = oracle.at_beta(raw, w["n"], p, ev.P, beta)
        ll, dcp = ev.loglik_adjoint(w["covparms"], beta)
        assert abs(float(ll.cpu()[0]) - at["loglik"]) <= 1e-10 * abs(at["loglik"])
        g = dcp.cpu().numpy()
        assert np.all(np.abs(g - at["grad"]) <= 1e-8 * np.maximum(np.abs(at["grad"]), sd)), \
            (m, beta, g, at["grad"])


@pytest.mark.parametrize("m,nu", [(33, 1.5), (45, 2.5), (60, 0.5)])
def test_kriging_weights_match_oracle(m, nu):
    w = _problem(500, m, V.FAMILY_ISO, nu, 2, seed=700 + m)
    ev = _ev(w)
    for i0, i1 in [(0, 500), (0, 1), (59, 61), (123, 444)]:
        _say(f"weights m={m} [{i0}, {i1})")
        got = ev.kriging_weights(w["covparms"], i0, i1).cpu().numpy()
        ref = oracle.kriging_weights(w["locs"], w["NN"], w["covparms"], w["family"], w["nu"], 0,
                                     i0, i1)
        np.testing.assert_allclose(got[:, :m], ref[:, :m], rtol=0, atol=1e-9)
        np.testing.assert_allclose(got[:, m], ref[:, m], rtol=0, atol=1e-10)


def test_kriging_predict_with_60_neighbours():
    m, p = 60, 3
    w = _problem(4000, m, V.FAMILY_ISO, 1.5, p, seed=777)
    rng = np.random.default_rng(778)
    npred = 1500
    lp = rng.random((npred, 2))
    Xp = np.column_stack([np.ones(npred)] + [rng.standard_normal(npred) for _ in range(p - 1)])
    NNp = S.nn_among(w["locs"], lp, m)
    ev = _ev(w)
    beta = ev.loglik(w["covparms"]).cpu().numpy()[1:1 + p]
    mean, var = V.Predictor(ev, lp, Xp, NNp).predict(w["covparms"], beta)
    ref_m, ref_v = oracle.kriging_predict(w["locs"], w["y"], w["X"], lp, Xp, NNp[:, 1:],
                                          w["covparms"], beta, w["family"], w["nu"])
    np.testing.assert_allclose(mean.cpu().numpy(), ref_m, rtol=1e-10,
                               atol=1e-10 * np.abs(ref_m).max())
    np.testing.assert_allclose(var.cpu().numpy(), ref_v, rtol=1e-10)


def test_ragged_tiles_and_tiny_problems():
    for n, m in [(1, 60), (2, 60), (61, 60), (62, 60), (1029, 60), (3, 45), (35, 34), (36, 32)]:
        w = _problem(n, m, V.FAMILY_ISO, 0.5, 1, seed=n + m)
        _say(f"tiny/ragged n={n} m={m}")
        raw, ref = _oracle(w)
        ev = _ev(w)
        got = V.unpack_out(ev.loglik_grad_info(w["covparms"]), 1, ev.P)
        _check(got, ref, f"n={n} m={m}")


def test_sweep_size_at_m60_sampled():
    """The size study's m = 60 configuration at n = 2^20 (2-D Matern 3/2,
    coarse-to-fine order, neighbours from the library's own search), in the
    launch the sweep times: sums over sampled observation ranges against the
    oracle."""
    n, m = 1 << 20, 60
    rng = np.random.default_rng(8)
    locs = rng.random((n, 2))
    locs = locs[S.maxmin_approx(locs, 8)]
    _say("m=60 sweep size: neighbours (the library's search, itself checked against brute force)")
    NN = V.ordered_nn(torch.as_tensor(np.ascontiguousarray(locs), device="cuda"), m).cpu().numpy()
    y = rng.standard_normal(n)
    X = np.ones((n, 1))
    cp = np.array((1.0, 0.05, 0.05))
    ev = V.Vecchia(locs, NN, y, X, V.FAMILY_ISO, 1.5, 0)
    for i0, i1 in [(0, 4096), (n // 2, n // 2 + 3001), (n - 2500, n)]:
        _say(f"m=60 sweep size: range [{i0}, {i1})")
        got = ev.raw_sums(cp, i0, i1).cpu().numpy()
        ref = oracle.raw_sums(locs, NN, y, X, cp, V.FAMILY_ISO, 1.5, 0, i0=i0, i1=i1, threads=8)
        g, r = oracle.unpack_raw(got, 1, 3), oracle.unpack_raw(ref, 1, 3)
        for key in r:
            a, b = np.asarray(g[key]), np.asarray(r[key])
            assert np.max(np.abs(a - b)) <= 1e-9 * max(np.max(np.abs(b)), 1e-300), (key, i0)

"""Parity cases beyond the main grid, through the C ABI:

* every split of the space-time coordinates (time not last runs on the
  wave-per-neighbourhood kernel; the entry points without it refuse);
* coincident locations with a nugget (h = 0 off the diagonal, where the
  range derivative is taken as 0) on both kernels;
* a prediction row naming another prediction point (reported, not used);
* the 262,144-point Matern 3/2 plane with p = 3 at full size: every raw sum
  against the oracle over every observation, and the adjoint gradient
  against the oracle's fixed-beta gradient and finite differences;
* the binding's shape checks (a Python error instead of a device read out
  of bounds).

Tolerances are those of test_gpu_parity.py.
"""

import os

import numpy as np
import pytest

import oracle
from paper_2407_02740_amd import synthetic as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from paper_2407_02740_amd import vecchia as V  # noqa: E402

from test_gpu_parity import check_outputs, check_raw  # noqa: E402


def _say(msg):
    print(msg, flush=True)


def _threads():
    return min(16, os.cpu_count() or 8)


def _run(locs, NN, y, X, cp, family, nu, nspace, tag):
    n, p = len(y), X.shape[1]
    _say(f"case {tag}: n={n} m={NN.shape[1] - 1} family={family} nspace={nspace}")
    ev = V.Vecchia(locs, NN, y, X, family, nu, nspace)
    got = V.unpack_out(ev.loglik_grad_info(cp), p, ev.P)
    got_raw = ev.raw.cpu().numpy()
    ref_raw = oracle.raw_sums(locs, NN, y, X, cp, family, nu, nspace, threads=8)
    ref = oracle.combine(ref_raw, n, p, ev.P)
    check_raw(got_raw, ref_raw, p, ev.P, tag)
    check_outputs(got, ref, tag)
    return ev


def _st_problem(n, d, nspace, m, seed, p=1):
    rng = np.random.default_rng(seed)
    locs = rng.random((n, d)) * np.array([1.0, 1.0, 1.0, 8.0])[:d]
    scale = np.array([0.3] * nspace + [2.0] * (d - nspace))
    locs = locs[S.maxmin_approx(locs / scale, seed)]
    NN = S.find_ordered_nn(locs / scale, m)
    y = rng.standard_normal(n) + 0.4 * np.sin(5 * locs[:, 0])
    X = np.column_stack([np.ones(n)] + [rng.standard_normal(n) for _ in range(p - 1)])
    return locs, NN, y, X, np.array((1.1, 0.3, 2.0, 0.1))


# ---------------------------------------------------------------------------
# space-time split
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d,nspace,m", [(2, 1, 30), (3, 1, 10), (3, 1, 30), (4, 1, 30),
                                        (4, 2, 20), (4, 3, 30), (4, 2, 50)])
def test_spacetime_every_coordinate_split(d, nspace, m):
    locs, NN, y, X, cp = _st_problem(3001, d, nspace, m, seed=500 + 10 * d + nspace, p=2)
    _run(locs, NN, y, X, cp, V.FAMILY_SPACETIME, 1.5, nspace, f"st d={d} nspace={nspace} m={m}")


def test_spacetime_split_off_the_fused_kernel_is_refused_where_unsupported():
    locs, NN, y, X, cp = _st_problem(500, 3, 1, 10, seed=7)
    ev = V.Vecchia(locs, NN, y, X, V.FAMILY_SPACETIME, 0.5, 1)
    with pytest.raises(V.VecchiaError) as e:
        ev.loglik(cp)
    assert e.value.code == V.VEC_EINVAL
    with pytest.raises(V.VecchiaError) as e:
        ev.loglik_adjoint(cp, [0.0])
    assert e.value.code == V.VEC_EINVAL
    with pytest.raises(V.VecchiaError) as e:
        ev.kriging_weights(cp)
    assert e.value.code == V.VEC_EINVAL
    # and the Fisher fit runs (wave kernel) and matches the oracle's
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        th = ev.covparms(cp * 1.2)
        ev.fisher_fit(th, 3, use_graph=True)
    torch.cuda.synchronize()
    th_ref, _ = oracle.fit(locs, NN, y, X, cp * 1.2, V.FAMILY_SPACETIME, 0.5, 1, iters=3)
    np.testing.assert_allclose(th.cpu().numpy(), th_ref, rtol=1e-8)


# ---------------------------------------------------------------------------
# coincident locations with a nugget
# ---------------------------------------------------------------------------
def _with_duplicates(locs, seed, frac=0.1):
    """Copies of earlier points placed at later positions of the ordering, so
    that a neighbourhood holds pairs at distance 0."""
    rng = np.random.default_rng(seed)
    n = len(locs)
    out = locs.copy()
    tgt = rng.choice(np.arange(n // 4, n), size=int(frac * n), replace=False)
    for t in tgt:
        out[t] = out[rng.integers(0, t)]
    return out


@pytest.mark.parametrize("family,nu,m,d,nspace", [(V.FAMILY_ISO, 0.5, 10, 2, 0),
                                                  (V.FAMILY_ISO, 1.5, 30, 2, 0),
                                                  (V.FAMILY_ISO, 2.5, 40, 2, 0),
                                                  (V.FAMILY_SPACETIME, 0.5, 30, 3, 2),
                                                  (V.FAMILY_SPACETIME, 1.5, 30, 4, 2),
                                                  (V.FAMILY_ISO, 0.5, 50, 2, 0),
                                                  (V.FAMILY_ANISO, 0.5, 30, 3, 0)])
def test_coincident_locations_with_nugget(family, nu, m, d, nspace):
    rng = np.random.default_rng(900 + m + d)
    n = 2500
    locs = rng.random((n, d))
    locs = locs[S.maxmin_approx(locs, 3)]
    locs = _with_duplicates(locs, 4)
    NN = S.find_ordered_nn(locs, m)
    # at least some neighbourhoods hold an exact twin
    twins = sum(np.any(np.all(locs[NN[i, 1:min(i, m) + 1]] == locs[i], axis=1))
                for i in range(1, n))
    assert twins > 50
    y = rng.standard_normal(n)
    X = np.ones((n, 1))
    cp = {V.FAMILY_ISO: (1.2, 0.2, 0.1), V.FAMILY_SPACETIME: (1.2, 0.3, 0.5, 0.1),
          V.FAMILY_ANISO: (1.2, 0.2, 0.4, 0.3, 0.1)}[family]
    _run(locs, NN, y, X, np.array(cp), family, nu, nspace,
         f"twins fam={family} nu={nu} m={m} d={d}")


# ---------------------------------------------------------------------------
# prediction rows may only name observed points
# ---------------------------------------------------------------------------
def test_prediction_row_naming_a_prediction_point_is_reported():
    rng = np.random.default_rng(77)
    n, m, npred = 2000, 10, 300
    locs = rng.random((n, 2))
    locs = locs[S.maxmin_approx(locs, 1)]
    NN = S.find_ordered_nn(locs, m)
    y = rng.standard_normal(n)
    X = np.ones((n, 1))
    ev = V.Vecchia(locs, NN, y, X, V.FAMILY_ISO, 0.5, 0)
    lp = rng.random((npred, 2))
    NNp = S.nn_among(locs, lp, m)
    cp = np.array((1.0, 0.2, 0.05))
    pr = V.Predictor(ev, lp, np.ones((npred, 1)), NNp)
    mean, _ = pr.predict(cp, [0.0])       # well formed: fine
    assert torch.isfinite(mean).all()
    bad = NNp.copy()
    bad[120, 3] = n + 5                   # another prediction point
    ev.clear_status()
    with pytest.raises(V.VecchiaError) as e:
        V.Predictor(ev, lp, np.ones((npred, 1)), bad).predict(cp, [0.0])
    assert e.value.code == V.VEC_EBADNN and e.value.bad_i == n + 120
    ev.clear_status()


# ---------------------------------------------------------------------------
# binding shape checks
# ---------------------------------------------------------------------------
def test_binding_rejects_mismatched_shapes():
    rng = np.random.default_rng(1)
    n, m = 200, 5
    locs = rng.random((n, 2))
    NN = S.find_ordered_nn(locs, m)
    y = rng.standard_normal(n)
    X = np.ones((n, 1))
    with pytest.raises(ValueError):
        V.Vecchia(locs, NN[:-1], y, X)
    with pytest.raises(ValueError):
        V.Vecchia(locs, NN, y[:-1], X)
    with pytest.raises(ValueError):
        V.Vecchia(locs, NN, y, X[:-3])
    ev = V.Vecchia(locs, NN, y, X)
    with pytest.raises(ValueError):
        ev.loglik_grad_info(torch.ones(4, dtype=torch.float64, device="cuda"))
    with pytest.raises(TypeError):
        ev.loglik_grad_info(torch.ones(3, dtype=torch.float32, device="cuda"))


# ---------------------------------------------------------------------------
# the Matern plane at full size (n = 262,144, Matern 3/2, p = 3)
# ---------------------------------------------------------------------------
@pytest.mark.skipif(os.environ.get("VECCHIA_SKIP_FULL") == "1", reason="full size skipped")
def test_full_size_matern_plane_forward_and_adjoint():
    _say("full-size matern plane: generating")
    w = S.matern_plane()
    n, p = w["n"], w["p"]
    cp = np.asarray(w["covparms"], dtype=float)
    threads = _threads()
    _say("full-size matern plane: GPU forward, loglik-only and adjoint")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ev = V.Vecchia(w["locs"], w["NN"], w["y"], w["X"], w["family"], w["nu"], w["nspace"])
        got = V.unpack_out(ev.loglik_grad_info(cp).clone(), p, ev.P)
        got_raw = ev.raw.cpu().numpy()
        lik = ev.loglik(cp).cpu().numpy()
    torch.cuda.synchronize()
    _say(f"full-size matern plane: oracle over all {n} observations on {threads} threads")
    ref_raw = oracle.raw_sums(w["locs"], w["NN"], w["y"], w["X"], cp, w["family"], w["nu"],
                              w["nspace"], threads=threads)
    ref = oracle.combine(ref_raw, n, p, ev.P)
    check_raw(got_raw, ref_raw, p, ev.P, "matern full")
    check_outputs(got, ref, "matern full")
    assert abs(lik[0] - ref["loglik"]) <= 1e-10 * abs(ref["loglik"])
    sd = np.sqrt(np.diag(ref["info"]))
    betas = (ref["betahat"], ref["betahat"] + np.array([0.3, -0.2, 0.1]))
    for k, beta in enumerate(betas):
        with torch.cuda.stream(stream):
            ll, dcp = ev.loglik_adjoint(cp, beta)
        torch.cuda.synchronize()
        at = oracle.at_beta(ref_raw, n, p, ev.P, beta)
        assert abs(float(ll.cpu()[0]) - at["loglik"]) <= 1e-10 * abs(at["loglik"])
        g = dcp.cpu().numpy()
        assert np.all(np.abs(g - at["grad"]) <= 1e-8 * np.maximum(np.abs(at["grad"]), sd)), \
            (k, g, at["grad"])
        if k == 1:
            # central differences of the oracle's log-likelihood at this fixed beta
            for j in range(ev.P):
                h = 1e-5 * cp[j]
                lo, hi = cp.copy(), cp.copy()
                lo[j] -= h
                hi[j] += h
                fl = [oracle.at_beta(oracle.raw_sums(w["locs"], w["NN"], w["y"], w["X"], c,
                                                     w["family"], w["nu"], w["nspace"],
                                                     threads=threads), n, p, ev.P,
                                     beta)["loglik"] for c in (hi, lo)]
                fd = (fl[0] - fl[1]) / (2 * h)
                _say(f"full-size matern plane: d/dtheta_{j} adjoint {g[j]:.9e} fd {fd:.9e}")
                assert abs(g[j] - fd) <= 1e-5 * max(abs(fd), sd[j])

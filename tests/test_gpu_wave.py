"""Parity of the wave-per-neighbourhood kernel with the CPU oracle, through
the C ABI, at the tolerances of test_gpu_parity: the one-range-per-coordinate
family on the full 18-attribute workload element by element and over a sweep
of dimensions, neighbour counts, covariates and smoothness values that spans
every kernel size (m + 1 <= 16, 32, 64) and coordinate block (d <= 4, 8, 16,
20, 32), with ragged first neighbourhoods (i < m); and the isotropic and
space-time families beyond the fused kernel's largest neighbourhood
(40 < m <= 63)."""

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

AN = V.FAMILY_ANISO


def _say(msg):
    print(msg, flush=True)


def _problem(n, d, m, p, nu, seed, tau2=0.08):
    rng = np.random.default_rng(seed)
    locs = rng.standard_normal((n, d))
    rho = np.exp(rng.uniform(np.log(0.5), np.log(4.0), d))
    NN = S.find_ordered_nn(locs / rho, m)
    y = rng.standard_normal(n) + 0.5 * np.sin(locs[:, 0])
    X = np.column_stack([np.ones(n)] + [rng.standard_normal(n) for _ in range(p - 1)])
    cp = np.concatenate([[1.2], rho, [tau2]])
    return dict(locs=locs, NN=NN, y=y, X=X, covparms=cp, family=AN, nu=nu, nspace=0, m=m, n=n,
                p=p, d=d)


def run_case(w, tag, threads=8, i0=0, i1=None):
    _say(f"case {tag}: n={w['n']} d={w['d']} m={w['m']} p={w['p']} nu={w['nu']}")
    ev = V.Vecchia(w["locs"], w["NN"], w["y"], w["X"], AN, w["nu"])
    assert ev.P == w["d"] + 2
    if i0 == 0 and i1 is None:
        got = V.unpack_out(ev.loglik_grad_info(w["covparms"]), w["p"], ev.P)
        got_raw = ev.raw.cpu().numpy()
        ref_raw = oracle.raw_sums(w["locs"], w["NN"], w["y"], w["X"], w["covparms"], AN, w["nu"],
                                  threads=threads)
        check_raw(got_raw, ref_raw, w["p"], ev.P, tag)
        check_outputs(got, oracle.combine(ref_raw, w["n"], w["p"], ev.P), tag)
    else:
        got_raw = ev.raw_sums(w["covparms"], i0, i1).cpu().numpy()
        ref_raw = oracle.raw_sums(w["locs"], w["NN"], w["y"], w["X"], w["covparms"], AN, w["nu"],
                                  i0=i0, i1=i1, threads=threads)
        check_raw(got_raw, ref_raw, w["p"], ev.P, tag)
    return ev


def test_attributes_18d_full_size():
    w = S.attributes_18d()
    run_case(w, "attributes_18d", threads=16)


@pytest.mark.parametrize("d,m,p,nu", [
    (1, 0, 1, 0.5), (1, 5, 2, 1.5), (3, 1, 1, 2.5), (5, 10, 3, 0.5), (8, 31, 1, 1.5),
    (9, 30, 2, 0.5), (16, 20, 1, 2.5), (17, 31, 3, 1.5), (18, 10, 1, 0.5), (24, 40, 1, 0.5),
    (32, 31, 2, 1.5), (32, 63, 1, 0.5), (7, 63, 3, 2.5), (12, 45, 2, 0.5)])
def test_shapes_match_the_oracle(d, m, p, nu):
    n = 1500 if m > 31 else 2500
    run_case(_problem(n, d, m, p, nu, seed=100 * d + m), f"d{d}m{m}p{p}")


@pytest.mark.parametrize("family,nu,m,p", [(0, 0.5, 60, 1), (0, 1.5, 45, 2), (1, 0.5, 60, 1),
                                           (1, 2.5, 63, 3)])
def test_isotropic_and_space_time_beyond_the_fused_sizes(family, nu, m, p):
    rng = np.random.default_rng(m + 10 * family)
    n = 3000
    d = 2 if family == 0 else 3
    locs = rng.random((n, d))
    locs = locs[S.maxmin_exact(locs)]
    cp = np.array((1.3, 0.15, 0.05)) if family == 0 else np.array((1.1, 0.3, 0.5, 0.1))
    scaled = locs / (cp[1] if family == 0 else np.array([cp[1], cp[1], cp[2]]))
    NN = S.find_ordered_nn(scaled, m)
    y = rng.standard_normal(n)
    X = np.column_stack([np.ones(n)] + [rng.standard_normal(n) for _ in range(p - 1)])
    _say(f"case family={family} nu={nu} m={m} p={p}")
    ev = V.Vecchia(locs, NN, y, X, family, nu, 2 if family == 1 else 0)
    got = V.unpack_out(ev.loglik_grad_info(cp), p, ev.P)
    ref_raw = oracle.raw_sums(locs, NN, y, X, cp, family, nu, nspace=2, threads=8)
    check_raw(ev.raw.cpu().numpy(), ref_raw, p, ev.P, f"m{m}")
    check_outputs(got, oracle.combine(ref_raw, n, p, ev.P), f"m{m}")


def test_tiny_inputs_and_ranges_of_observations():
    run_case(_problem(1, 4, 10, 1, 0.5, 1), "n1")
    run_case(_problem(7, 4, 10, 2, 1.5, 2), "n7<m")
    w = _problem(3000, 18, 30, 1, 0.5, 3)
    for i0, i1 in [(0, 17), (5, 31), (1000, 2999), (2999, 3000), (40, 40)]:
        run_case(w, f"range{i0}-{i1}", i0=i0, i1=i1)


def test_equal_ranges_match_the_isotropic_kernel():
    # the two kernels share no code; with every range equal the anisotropic
    # sums collapse to the isotropic ones (range entries add up)
    rng = np.random.default_rng(8)
    n, m, d = 4000, 30, 3
    locs = rng.random((n, d))
    locs = locs[S.maxmin_approx(locs, 8)]
    NN = S.find_ordered_nn(locs, m)
    y = rng.standard_normal(n)
    X = np.ones((n, 1))
    a = V.Vecchia(locs, NN, y, X, AN, 1.5)
    b = V.Vecchia(locs, NN, y, X, V.FAMILY_ISO, 1.5)
    ra = V.unpack_out(a.loglik_grad_info([1.1, 0.2, 0.2, 0.2, 0.05]), 1, 5)
    rb = V.unpack_out(b.loglik_grad_info([1.1, 0.2, 0.05]), 1, 3)
    assert abs(ra["loglik"] - rb["loglik"]) <= 1e-10 * abs(rb["loglik"])
    C = np.zeros((3, 5))
    C[0, 0] = C[2, 4] = 1.0
    C[1, 1:4] = 1.0
    np.testing.assert_allclose(C @ ra["grad"], rb["grad"], rtol=1e-8, atol=1e-8)
    np.testing.assert_allclose(C @ ra["info"] @ C.T, rb["info"], rtol=1e-9)


def test_fisher_scoring_matches_the_oracle():
    w = _problem(3000, 6, 15, 1, 0.5, 4)
    start = w["covparms"] * np.r_[1.5, np.full(6, 0.7), 2.0]
    ev = V.Vecchia(w["locs"], w["NN"], w["y"], w["X"], AN, 0.5)
    cp = torch.as_tensor(start, device="cuda")
    for use_graph in (False, True):
        cp.copy_(torch.as_tensor(start))
        ev.fisher_fit(cp, 3, use_graph=use_graph)
        got = cp.cpu().numpy()
        ref, _ = oracle.fit(w["locs"], w["NN"], w["y"], w["X"], start, AN, 0.5, iters=3,
                            threads=8)
        np.testing.assert_allclose(got, ref, rtol=1e-8)


def test_errors_are_flagged():
    w = _problem(500, 5, 8, 1, 0.5, 5)
    NN = w["NN"].copy()
    NN[123, 3] = 200  # not a previous observation
    ev = V.Vecchia(w["locs"], NN, w["y"], w["X"], AN, 0.5)
    with pytest.raises(V.VecchiaError) as e:
        ev.loglik_grad_info(w["covparms"])
    assert e.value.code == V.VEC_EBADNN and e.value.bad_i == 123
    # a negative nugget ratio: the first neighbourhood whose covariance is
    # indefinite is the one the oracle stops at
    cp = w["covparms"].copy()
    cp[-1] = -0.6
    with pytest.raises(oracle.OracleError) as eo:
        oracle.raw_sums(w["locs"], w["NN"], w["y"], w["X"], cp, AN, 0.5)
    ev = V.Vecchia(w["locs"], w["NN"], w["y"], w["X"], AN, 0.5)
    with pytest.raises(V.VecchiaError) as e:
        ev.loglik_grad_info(cp)
    assert e.value.code == V.VEC_ENOTPD and e.value.bad_i == eo.value.bad_i
    # entry points other than the loglik/gradient/Fisher sums refuse the family
    ev = V.Vecchia(w["locs"], w["NN"], w["y"], w["X"], AN, 0.5)
    with pytest.raises(V.VecchiaError) as e:
        ev.loglik(w["covparms"])
    assert e.value.code == V.VEC_EINVAL

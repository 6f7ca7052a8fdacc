"""Grouped Vecchia on the device (vec_grouped_*) against the grouped oracle
(block conditionals, oracle/grouped.py) at the tolerances of
test_gpu_parity, through the C ABI: blocks from the host grid grouping on
2-D, space-time and anisotropic problems, blocks of one observation against
the single-observation path, full conditioning against the exact GP, Fisher
scoring, and malformed blocks."""

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


def _grouped_problem(n, d, g, m, family, seed, p=1):
    rng = np.random.default_rng(seed)
    locs = rng.random((n, d))
    order, bs, cs, cond = S.group_cells(locs, g, m, seed=seed)
    locs = locs[order]
    y = rng.standard_normal(n) + 0.4 * np.sin(5 * locs[:, 0])
    X = np.column_stack([np.ones(n)] + [rng.standard_normal(n) for _ in range(p - 1)])
    cp = {0: np.array((1.3, 0.12, 0.05)), 1: np.array((1.1, 0.2, 0.4, 0.08)),
          2: np.concatenate([[1.2], np.linspace(0.1, 0.3, d), [0.06]])}[family]
    return locs, y, X, cp, bs, cs, cond


def _run(locs, y, X, cp, bs, cs, cond, family, nu, tag, nspace=0):
    _say(f"case {tag}: n={len(y)} blocks={len(bs) - 1} family={family} nu={nu}")
    ev = V.GroupedVecchia(locs, y, X, bs, cs, cond, family, nu, nspace)
    got = V.unpack_out(ev.loglik_grad_info(cp), X.shape[1], ev.P)
    ref_raw = oracle.grouped_raw_sums(locs, y, X, cp, bs, cs, cond, family, nu, nspace)
    check_raw(ev.raw.cpu().numpy(), ref_raw, X.shape[1], ev.P, tag)
    check_outputs(got, oracle.combine(ref_raw, len(y), X.shape[1], ev.P), tag)
    return ev


@pytest.mark.parametrize("g,m,nu,p", [(4, 30, 0.5, 1), (8, 20, 1.5, 2), (2, 40, 2.5, 1),
                                      (8, 56, 0.5, 3)])
def test_isotropic_blocks_match_the_oracle(g, m, nu, p):
    prob = _grouped_problem(12_000, 2, g, m, 0, seed=g * 100 + m, p=p)
    _run(*prob, 0, nu, f"iso g{g} m{m}")


def test_space_time_and_anisotropic_blocks():
    locs, y, X, cp, bs, cs, cond = _grouped_problem(8000, 3, 6, 25, 1, seed=7)
    _run(locs, y, X, cp, bs, cs, cond, 1, 0.5, "space-time", nspace=2)
    locs, y, X, cp, bs, cs, cond = _grouped_problem(8000, 4, 4, 30, 2, seed=8)
    _run(locs, y, X, cp, bs, cs, cond, 2, 1.5, "anisotropic d4")


def test_blocks_of_one_are_the_single_observation_path():
    rng = np.random.default_rng(9)
    n, m, d = 6000, 30, 18
    locs = rng.standard_normal((n, d))
    NN = S.find_ordered_nn(locs, m)
    y = rng.standard_normal(n)
    X = np.ones((n, 1))
    cp = np.concatenate([[1.0], np.full(d, 3.0), [0.1]])
    rows = [NN[i, 1:1 + min(i, m)] for i in range(n)]
    cs = np.r_[0, np.cumsum([len(r) for r in rows])]
    cond = np.concatenate(rows).astype(np.int32)
    ev = V.GroupedVecchia(locs, y, X, np.arange(n + 1), cs, cond, V.FAMILY_ANISO, 0.5)
    a = ev.raw_sums(cp).cpu().numpy()
    b = V.Vecchia(locs, NN, y, X, V.FAMILY_ANISO, 0.5).raw_sums(cp).cpu().numpy()
    ref = oracle.raw_sums(locs, NN, y, X, cp, V.FAMILY_ANISO, 0.5, threads=8)
    check_raw(a, ref, 1, d + 2, "blocks of one")
    check_raw(b, ref, 1, d + 2, "single path")


def test_full_conditioning_is_the_exact_gp():
    rng = np.random.default_rng(10)
    n = 40
    locs = rng.random((n, 2))
    y = rng.standard_normal(n)
    X = np.ones((n, 1))
    cp = np.array((1.2, 0.3, 0.1))
    bs = np.array([0, 8, 16, 24, 32, 40])
    cs = np.r_[0, np.cumsum([0, 8, 16, 24, 32])]
    cond = np.concatenate([np.arange(k) for k in (0, 8, 16, 24, 32)]).astype(np.int32)
    ev = V.GroupedVecchia(locs, y, X, bs, cs, cond, 0, 0.5)
    got = V.unpack_out(ev.loglik_grad_info(cp), 1, 3)
    S_, dS = oracle.cov_matrix(locs, cp, 0, 0.5)
    Si = np.linalg.inv(S_)
    one = np.ones(n)
    beta = (one @ Si @ y) / (one @ Si @ one)
    r = y - beta
    ll = -0.5 * (n * np.log(2 * np.pi) + np.linalg.slogdet(S_)[1] + r @ Si @ r)
    assert abs(got["loglik"] - ll) <= 1e-10 * abs(ll)
    info = np.array([[0.5 * np.trace(Si @ dS[j] @ Si @ dS[k]) for k in range(3)] for j in range(3)])
    np.testing.assert_allclose(got["info"], info, rtol=1e-8)


def test_fisher_scoring_matches_the_oracle():
    locs, y, X, cp, bs, cs, cond = _grouped_problem(5000, 2, 4, 20, 0, seed=11)
    start = cp * np.array([1.6, 0.6, 2.5])
    ev = V.GroupedVecchia(locs, y, X, bs, cs, cond, 0, 1.5)
    th = start.copy()
    for _ in range(3):
        raw = oracle.grouped_raw_sums(locs, y, X, th, bs, cs, cond, 0, 1.5)
        res = oracle.combine(raw, len(y), 1, 3)
        th = oracle.fisher_step(th, res["grad"], res["info"])
    for use_graph in (False, True):
        t = torch.as_tensor(start, device="cuda")
        ev.fisher_fit(t, 3, use_graph=use_graph)
        np.testing.assert_allclose(t.cpu().numpy(), th, rtol=1e-8)


def test_malformed_blocks_and_empty_input():
    locs, y, X, cp, bs, cs, cond = _grouped_problem(3000, 2, 4, 10, 0, seed=12)
    bad = cond.copy()
    b = 500
    bad[cs[b]] = bs[b] + 1  # not an earlier observation
    ev = V.GroupedVecchia(locs, y, X, bs, cs, bad, 0, 0.5)
    with pytest.raises(V.VecchiaError) as e:
        ev.raw_sums(cp)
    assert e.value.code == V.VEC_EBADNN and e.value.bad_i == bs[b]
    # a conditioning set longer than the problem's m is refused on the device
    ev = V.GroupedVecchia(locs, y, X, bs, cs, cond, 0, 0.5)
    ev.pb.m = 5
    with pytest.raises(V.VecchiaError) as e:
        ev.raw_sums(cp)
    assert e.value.code == V.VEC_EBADNN
    # no blocks: zero sums
    ev = V.GroupedVecchia(locs, y, X, [0], [0], [], 0, 0.5)
    assert float(ev.raw_sums(cp).abs().sum()) == 0.0


def test_full_size_plane_sampled_blocks():
    """The grouped benchmark problem at its full size (n = 262,144 points of
    the plane, blocks of at most 4, m = 30, Matern 3/2), as the benchmark
    groups it: the sums over two ranges of its blocks (the first ones, whose
    conditioning sets are still short, and late ones), each launched like the
    full problem (more blocks than the 8 workgroups per CU of the grid)."""
    n, m, g = 262_144, 30, 4
    rng = np.random.default_rng(21)
    locs = rng.random((n, 2))
    order, bs, cs, cond = S.group_cells(locs, g, m, seed=21)
    pts = locs[order]
    y = rng.standard_normal(n)
    X = np.column_stack([np.ones(n), rng.standard_normal(n)])
    cp = np.array((1.0, 0.05, 0.05))
    nb = len(bs) - 1
    for b0, b1 in ((0, 2200), (nb - 2300, nb)):
        sbs = bs[b0:b1 + 1]
        scs = cs[b0:b1 + 1] - cs[b0]
        scond = cond[cs[b0]:cs[b1]]
        _say(f"case blocks [{b0}, {b1}) of {nb}")
        ev = V.GroupedVecchia(pts, y, X, sbs, scs, scond, 0, 1.5)
        got = ev.raw_sums(cp).cpu().numpy()
        ref = oracle.grouped_raw_sums(pts, y, X, cp, sbs, scs, scond, 0, 1.5)
        check_raw(got, ref, 2, ev.P, f"blocks {b0}-{b1}")

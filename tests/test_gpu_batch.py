"""Parity of the batched persistent path (many datasets of uneven n and m in
work-queue launches) with the CPU oracle, dataset by dataset, through the C
ABI.  Tolerances as in test_gpu_parity.
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


def _say(msg):
    print(msg, flush=True)


def check_outputs(got: dict, ref: dict, tag=""):
    assert abs(got["loglik"] - ref["loglik"]) <= 1e-10 * abs(ref["loglik"]), \
        (tag, got["loglik"], ref["loglik"])
    I = ref["info"]
    sd = np.sqrt(np.abs(np.diag(I)))
    assert np.all(np.abs(got["grad"] - ref["grad"]) <= 1e-8 * np.maximum(np.abs(ref["grad"]), sd)), \
        (tag, got["grad"], ref["grad"])
    assert np.all(np.abs(got["info"] - I) <= 1e-8 * np.maximum(np.abs(I), np.outer(sd, sd))), \
        (tag, got["info"], I)
    bscale = np.abs(ref["betahat"]) + 1.0 / np.sqrt(np.diag(ref["betainfo"]))
    assert np.all(np.abs(got["betahat"] - ref["betahat"]) <= 1e-8 * bscale), tag


def _vb(w, sched=None, NN=None):
    return V.VecchiaBatch(w["locs"], w["NN"] if NN is None else NN, w["y"], w["X"],
                          w["obs_offset"], w["nn_offset"], w["n"], w["m"], w["nu"],
                          w["family"], w["nspace"], sched=sched)


def _oracle_member(w, b, covparms=None):
    d = S.batch_member(w, b)
    cp = d["covparms"] if covparms is None else covparms
    return oracle.loglik_grad_info(d["locs"], d["NN"], d["y"], d["X"], cp, d["family"], d["nu"],
                                   d["nspace"], threads=8)


def _small_batch(nsets=24, n_min=300, n_max=6000, seed=40, ms=(10, 20, 30, 40)):
    return S.batched_uneven(seed=seed, nsets=nsets, n_min=n_min, n_max=n_max, ms=ms, workers=8)


@pytest.mark.parametrize("tile", [1, 7, 32, 1000])
def test_batch_matches_oracle_per_dataset(tile):
    w = _small_batch()
    _say(f"batch of {w['nsets']} datasets, tile {tile}, classes {np.bincount(w['m'] // 10)}")
    vb = _vb(w, V.schedule(tile=tile))
    out = vb.loglik_grad_info(w["covparms"]).cpu().numpy()
    for b in range(w["nsets"]):
        ref = _oracle_member(w, b)
        check_outputs(V.unpack_out(out[b], 1, vb.P), ref, f"dataset {b} n={w['n'][b]} m={w['m'][b]}")


def test_batch_edge_cases():
    """n = 1, n <= m, m = 0, a single class, one dataset."""
    rng = np.random.default_rng(41)
    parts = []
    for n, m, nu in [(1, 0, 0.5), (1, 10, 1.5), (5, 40, 2.5), (41, 40, 0.5), (3000, 0, 1.5),
                     (700, 40, 0.5), (17, 3, 2.5)]:
        locs = rng.random((n, 2))
        locs = locs[S.maxmin_exact(locs)]
        parts.append((locs, S.find_ordered_nn(locs, m), rng.standard_normal(n), m, nu,
                      (1.2, 0.1, 0.05)))
    n = np.array([len(p[2]) for p in parts])
    m = np.array([p[3] for p in parts])
    w = dict(locs=np.concatenate([p[0] for p in parts]),
             NN=np.concatenate([p[1].reshape(-1) for p in parts]).astype(np.int32),
             y=np.concatenate([p[2] for p in parts]), X=np.ones((n.sum(), 1)), n=n, m=m,
             obs_offset=np.concatenate([[0], np.cumsum(n)[:-1]]),
             nn_offset=np.concatenate([[0], np.cumsum(n * (m + 1))[:-1]]),
             nu=np.array([p[4] for p in parts]), covparms=np.array([p[5] for p in parts]),
             family=V.FAMILY_ISO, nspace=0, nsets=len(parts), name="edge")
    for sel in (list(range(len(parts))), [4], [1, 2, 3, 5]):
        sub = {**w, "n": n[sel], "m": m[sel], "obs_offset": w["obs_offset"][sel],
               "nn_offset": w["nn_offset"][sel], "nu": w["nu"][sel],
               "covparms": w["covparms"][sel], "nsets": len(sel)}
        vb = _vb(sub, V.schedule(tile=16))
        out = vb.loglik_grad_info(sub["covparms"]).cpu().numpy()
        for j, b in enumerate(sel):
            check_outputs(V.unpack_out(out[j], 1, vb.P), _oracle_member(w, b), f"edge {b}")


def test_batch_is_deterministic_and_matches_single_problem_path():
    w = _small_batch(nsets=16, seed=42)
    vb = _vb(w)
    a = vb.loglik_grad_info(w["covparms"]).clone()
    b = vb.loglik_grad_info(w["covparms"]).clone()
    assert torch.equal(a, b)
    out = a.cpu().numpy()
    for k in range(0, w["nsets"], 5):
        d = S.batch_member(w, k)
        ev = V.Vecchia(d["locs"], d["NN"], d["y"], d["X"], d["family"], d["nu"], d["nspace"])
        single = V.unpack_out(ev.loglik_grad_info(d["covparms"]), 1, ev.P)
        check_outputs(V.unpack_out(out[k], 1, vb.P), single, f"single {k}")


def test_batch_errors_are_per_dataset():
    w = _small_batch(nsets=6, seed=43, n_min=1000, n_max=3000)
    NN = w["NN"].copy()
    b = 2
    o, mb = int(w["nn_offset"][b]), int(w["m"][b])
    row = 500
    NN[o + row * (mb + 1) + 1] = row + 3   # a neighbour that does not precede its row
    vb = _vb(w, NN=NN)
    vb.loglik_grad_info(w["covparms"], check=False)
    torch.cuda.synchronize()
    codes = vb.status_codes()
    assert codes[b] == V.VEC_EBADNN and int(vb.status[b, 1]) == row
    assert all(c == V.VEC_OK for k, c in enumerate(codes) if k != b)
    out = vb.out.cpu().numpy()
    for k in (0, 5):
        check_outputs(V.unpack_out(out[k], 1, vb.P), _oracle_member(w, k), f"healthy {k}")


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_fisher_fit_matches_oracle(use_graph):
    w = _small_batch(nsets=5, seed=44, n_min=1500, n_max=3000, ms=(10, 20))
    start = w["covparms"] * np.array([0.8, 1.4, 1.5])
    iters = 4
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        vb = _vb(w)
        cp = vb.covparms(start)
        vb.fisher_fit(cp, iters, use_graph=use_graph)
    torch.cuda.synchronize()
    got = cp.cpu().numpy()
    for b in range(w["nsets"]):
        d = S.batch_member(w, b)
        th, _ = oracle.fit(d["locs"], d["NN"], d["y"], d["X"], start[b], d["family"], d["nu"],
                           d["nspace"], iters=iters, threads=8)
        np.testing.assert_allclose(got[b], th, rtol=1e-8, err_msg=f"dataset {b}")


@pytest.mark.skipif(os.environ.get("VECCHIA_SKIP_FULL") == "1", reason="full size skipped")
def test_full_size_batched_uneven():
    """512 datasets, about 1.3e7 neighbourhoods, in the benchmark's launch
    configuration: 32 sampled datasets (eight of every size class, its
    smallest and largest among them) against the oracle, every dataset
    against the single-problem kernel (itself checked against the oracle at
    full size)."""
    _say("full batched: generating")
    w = S.batched_uneven()
    _say(f"full batched: {w['nsets']} datasets, {int(w['n'].sum())} observations")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        vb = _vb(w)
        out = vb.loglik_grad_info(w["covparms"]).cpu().numpy()
    torch.cuda.synchronize()
    # per size class: its smallest and largest dataset and six more drawn
    # with a fixed seed (32 of the 512 against the oracle)
    rng = np.random.default_rng(149)
    picks = []
    for m in (10, 20, 30, 40):
        members = np.flatnonzero(w["m"] == m)
        by_n = members[np.argsort(w["n"][members], kind="stable")]
        extra = rng.choice(by_n[1:-1], size=min(6, len(by_n) - 2), replace=False)
        picks += [int(by_n[0]), int(by_n[-1])] + [int(b) for b in extra]
    for b in picks:
        _say(f"full batched: oracle on dataset {b} (n={w['n'][b]}, m={w['m'][b]})")
        check_outputs(V.unpack_out(out[b], 1, vb.P), _oracle_member(w, b), f"full {b}")
    _say("full batched: single-problem kernel on every dataset")
    for b in range(w["nsets"]):
        d = S.batch_member(w, b)
        ev = V.Vecchia(d["locs"], d["NN"], d["y"], d["X"], d["family"], d["nu"], d["nspace"])
        single = V.unpack_out(ev.loglik_grad_info(d["covparms"]), 1, ev.P)
        check_outputs(V.unpack_out(out[b], 1, vb.P), single, f"single {b}")


def test_autotuner_picks_a_measured_schedule_and_stays_exact():
    """The tuner times each size class under every candidate, keeps the
    fastest, and the batch evaluated under the chosen plan still matches the
    oracle dataset by dataset."""
    import paper_2407_02740_amd.autotune as AT

    w = _small_batch(nsets=12, seed=45, n_min=2000, n_max=5000)
    vb = _vb(w)
    sched, table = AT.tune_batch(vb, w["covparms"], tiles=(8, 64), blocks=(0,), reps=2, log=_say)
    present = {min(c for c, K in enumerate(V.CLASS_K) if m + 1 <= K) for m in w["m"]}
    assert set(table) == present
    for c, rows in table.items():
        assert len(rows) == 2 and all(ms > 0 for _, _, ms in rows)
        best = min(rows, key=lambda r: r[2])
        assert sched.tile[c] == best[0] and vb.plan.sched.tile[c] == best[0]
    out = vb.loglik_grad_info(w["covparms"]).cpu().numpy()
    for b in range(w["nsets"]):
        check_outputs(V.unpack_out(out[b], 1, vb.P), _oracle_member(w, b), f"tuned {b}")

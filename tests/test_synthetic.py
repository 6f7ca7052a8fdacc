"""Host-side input generators: ordering, neighbour arrays, seeding."""

import numpy as np

from paper_2407_02740_amd import synthetic as S


def test_maxmin_exact_picks_farthest_point_each_step():
    rng = np.random.default_rng(0)
    locs = rng.random((300, 2))
    order = S.maxmin_exact(locs)
    assert sorted(order) == list(range(300))
    pts = locs[order]
    for k in range(1, 60):
        d_prev = np.sqrt(((pts[k:, None] - pts[None, :k]) ** 2).sum(-1)).min(1)
        assert d_prev[0] >= d_prev.max() - 1e-12


def test_maxmin_approx_is_a_coarse_to_fine_permutation():
    rng = np.random.default_rng(1)
    locs = rng.random((20_000, 2))
    order = S.maxmin_approx(locs, 0)
    assert np.array_equal(np.sort(order), np.arange(20_000))
    pts = locs[order]
    # the first 64 points spread out far more than 64 random points do
    d_first = np.sqrt(((pts[:64, None] - pts[None, :64]) ** 2).sum(-1))
    np.fill_diagonal(d_first, np.inf)
    d_rand = np.sqrt(((locs[:64, None] - locs[None, :64]) ** 2).sum(-1))
    np.fill_diagonal(d_rand, np.inf)
    assert d_first.min() > 2 * d_rand.min()


def _coarse_to_fine_by_definition(locs, tie):
    """The ordering written out point by point: grid cell, bit-reversed
    interleaved code, rank in the cell by (tie, index), then one Python sort
    of (rank, code, tie, index) tuples."""
    n, d = locs.shape
    B = min(max(1, int(np.ceil(np.log2(max(n, 2)) / d))), 60 // d)
    lo, hi = locs.min(0), locs.max(0)
    keys = []
    for i in range(n):
        bits = []
        for b in range(B - 1, -1, -1):
            for k in range(d):
                span = max(hi[k] - lo[k], 1e-300)
                c = min(int((locs[i, k] - lo[k]) / span * 2 ** B), 2 ** B - 1)
                bits.append((c >> b) & 1)
        # bit-reversed: the first interleaved bit is the least significant
        rev = sum(bit << j for j, bit in enumerate(bits))
        keys.append((rev, tie[i], i))
    by_cell = sorted(keys)
    rank = {}
    for pos, (rev, t, i) in enumerate(by_cell):
        rank[i] = 0 if pos == 0 or by_cell[pos - 1][0] != rev else rank[by_cell[pos - 1][2]] + 1
    return np.array([i for _, _, _, i in sorted((rank[i], r, t, i) for r, t, i in keys)])


def test_maxmin_approx_follows_its_definition():
    rng = np.random.default_rng(7)
    for n, d in [(1, 2), (2, 1), (300, 1), (500, 2), (700, 3)]:
        locs = rng.random((n, d))
        tie = rng.random(n)
        assert np.array_equal(S.maxmin_approx(locs, tie=tie), _coarse_to_fine_by_definition(locs, tie))
    # clustered points (many per cell), repeated ties and a zero-extent axis
    locs = np.column_stack([rng.integers(0, 4, 400) / 4.0, np.zeros(400)])
    tie = rng.integers(0, 3, 400).astype(float)
    assert np.array_equal(S.maxmin_approx(locs, tie=tie), _coarse_to_fine_by_definition(locs, tie))


def test_ordered_nn_matches_brute_force():
    rng = np.random.default_rng(2)
    for d in (2, 4):
        locs = rng.random((1500, d))
        m = 12
        NN = S.find_ordered_nn(locs, m)
        assert NN.dtype == np.int32 and NN.shape == (1500, m + 1)
        assert np.array_equal(NN[:, 0], np.arange(1500))
        for i in list(range(0, 40)) + list(range(40, 1500, 37)):
            q = min(i, m)
            assert np.all(NN[i, q + 1:] == -1)
            nb = NN[i, 1:q + 1]
            assert np.all((nb >= 0) & (nb < i))
            dist = ((locs[:i] - locs[i]) ** 2).sum(1)
            ref = np.sort(dist)[:q]
            np.testing.assert_allclose(np.sort(dist[nb]), ref, rtol=1e-12)


def test_workloads_are_seeded_and_shaped():
    a = S.small_exponential(n=300, m=10)
    b = S.small_exponential(n=300, m=10)
    assert np.array_equal(a["y"], b["y"]) and np.array_equal(a["NN"], b["NN"])
    assert a["locs"].shape == (300, 2) and a["X"].shape == (300, 1)
    c = S.matern_plane(n=3000, m=30)
    assert c["X"].shape == (3000, 3) and len(np.unique(c["locs"], axis=0)) == 3000
    s = S.satellite_spacetime(slices=4, passes=4, per_pass=64, m=30)
    assert s["locs"].shape == (1024, 4) and s["nspace"] == 3
    xyz = s["locs"][:, :3]
    np.testing.assert_allclose((xyz ** 2).sum(1), 1.0, rtol=1e-12)
    lat = np.degrees(np.arcsin(xyz[:, 2]))
    assert np.abs(lat).max() <= 60.0 + 1e-9


def test_batched_uneven_offsets_and_worker_independence():
    a = S.batched_uneven(seed=9, nsets=6, n_min=300, n_max=900, workers=1)
    b = S.batched_uneven(seed=9, nsets=6, n_min=300, n_max=900, workers=3)
    for k in ("locs", "NN", "y", "n", "m", "covparms", "nu"):
        np.testing.assert_array_equal(a[k], b[k])
    n, m = a["n"], a["m"]
    assert a["locs"].shape == (n.sum(), 2) and a["NN"].size == int((n * (m + 1)).sum())
    assert np.all(np.isin(m, [10, 20, 30, 40]))
    for bi in range(6):
        d = S.batch_member(a, bi)
        NN = d["NN"]
        assert NN.shape == (n[bi], m[bi] + 1)
        assert np.all(NN[:, 0] == np.arange(n[bi]))
        valid = NN[:, 1:] >= 0
        assert np.all(NN[:, 1:][valid] < np.arange(n[bi])[:, None].repeat(m[bi], 1)[valid])
        assert 0.02 <= d["covparms"][1] <= 0.3 and 0.01 <= d["covparms"][2] <= 0.5


def test_surrogate_plane_shape():
    w = S.surrogate_plane(n=2000)
    assert w["NN"].shape == (2000, 31) and w["locs"].shape == (2000, 2)
    assert tuple(w["covparms"]) == (1.0, 0.05, 0.05) and w["nu"] == 1.5


def test_nn_among_lists_the_nearest_observed_points():
    rng = np.random.default_rng(3)
    obs = rng.random((500, 2))
    pred = rng.random((20, 2))
    NN = S.nn_among(obs, pred, 7)
    assert NN.shape == (20, 8) and np.all(NN[:, 0] == 500 + np.arange(20))
    for j in range(20):
        d = ((obs - pred[j]) ** 2).sum(1)
        np.testing.assert_array_equal(NN[j, 1:], np.argsort(d, kind="stable")[:7])

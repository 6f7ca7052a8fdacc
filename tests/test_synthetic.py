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

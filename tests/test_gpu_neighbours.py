"""The device neighbour search against brute force (its definition) and
against the host k-d tree search of the input module, bit-exact on the
indices (continuous random coordinates have no ties)."""

import numpy as np
import pytest

from paper_2407_02740_amd import synthetic as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from paper_2407_02740_amd import vecchia as V  # noqa: E402


def brute(locs, m):
    n = len(locs)
    NN = np.full((n, m + 1), -1, dtype=np.int32)
    NN[:, 0] = np.arange(n)
    for i in range(1, n):
        d = ((locs[:i] - locs[i]) ** 2).sum(1)
        o = np.lexsort((np.arange(i), d))[:min(i, m)]
        NN[i, 1:1 + len(o)] = o
    return NN


@pytest.mark.parametrize("d", [1, 2, 3, 4])
@pytest.mark.parametrize("m", [0, 1, 5, 30, 40])
def test_brute_force_small(d, m):
    rng = np.random.default_rng(10 * d + m)
    locs = rng.random((1500, d)) * np.array([1.0, 3.0, 0.5, 2.0][:d])
    locs = locs[S.maxmin_exact(locs)]
    got = V.ordered_nn(locs, m).cpu().numpy()
    np.testing.assert_array_equal(got, brute(locs, m))


def test_degenerate_and_tiny_inputs():
    # points on a line in 3-D (two dimensions of zero extent), n < m, n = 1
    rng = np.random.default_rng(3)
    t = rng.random(700)
    locs = np.column_stack([t, np.zeros(700), np.full(700, 2.0)])
    np.testing.assert_array_equal(V.ordered_nn(locs, 12).cpu().numpy(), brute(locs, 12))
    small = rng.random((9, 2))
    np.testing.assert_array_equal(V.ordered_nn(small, 20).cpu().numpy(), brute(small, 20))
    np.testing.assert_array_equal(V.ordered_nn(small[:1], 4).cpu().numpy(), brute(small[:1], 4))


@pytest.mark.parametrize("n,m", [(100_000, 30), (262_144, 10)])
def test_matches_the_host_search(n, m):
    rng = np.random.default_rng(n + m)
    locs = rng.random((n, 2))
    locs = locs[S.maxmin_approx(locs, 1)]
    got = V.ordered_nn(locs, m).cpu().numpy()
    ref = S.find_ordered_nn(locs, m)
    np.testing.assert_array_equal(got, ref)


def test_space_time_scaled_3d():
    w = S.satellite_spacetime(slices=2, passes=8, per_pass=256, m=30)
    scaled = w["locs"][:, :3] / 0.0872388
    got = V.ordered_nn(scaled, 30).cpu().numpy()
    np.testing.assert_array_equal(got, S.find_ordered_nn(scaled, 30))


@pytest.mark.parametrize("d,m", [(4, 0), (4, 10), (7, 1), (18, 30), (32, 64), (9, 40)])
def test_exhaustive_search_in_more_dimensions(d, m):
    rng = np.random.default_rng(100 + d + m)
    locs = rng.standard_normal((1200, d)) * np.linspace(0.5, 2.0, d)
    got = V.ordered_nn(locs, m).cpu().numpy()
    np.testing.assert_array_equal(got, brute(locs, m))


def test_attribute_workload_neighbours():
    # the 18-attribute workload: neighbours in range-scaled coordinates
    w = S.attributes_18d()
    rho = w["covparms"][1:-1]
    got = V.ordered_nn(w["locs"] / rho, w["m"]).cpu().numpy()
    np.testing.assert_array_equal(got, w["NN"])


def test_space_time_scaled_4d_matches_the_host_search():
    # the space-time workload's neighbour search: unit-sphere xyz / rho_s and
    # time / rho_t, in the coarse-to-fine order
    rng = np.random.default_rng(17)
    lon, lat, t = S.satellite_tracks(16, 64, 256, rng)
    la, lo = np.radians(lat), np.radians(lon)
    xyz = np.column_stack([np.cos(la) * np.cos(lo), np.cos(la) * np.sin(lo), np.sin(la)])
    scaled = np.column_stack([xyz / S.RHO_SPACE_5DEG, t / 3.0])
    scaled = np.ascontiguousarray(scaled[S.maxmin_approx(scaled, 17)])
    got = V.ordered_nn(scaled, 30).cpu().numpy()
    np.testing.assert_array_equal(got, S.find_ordered_nn(scaled, 30))

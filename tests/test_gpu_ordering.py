"""The device coarse-to-fine ordering against the host one of the input
module (itself pinned to a point-by-point definition in test_synthetic),
bit-exact on the permutation, with the same tie keys."""

import numpy as np
import pytest

from paper_2407_02740_amd import synthetic as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from paper_2407_02740_amd import vecchia as V  # noqa: E402


def check(locs, tie):
    order, out = V.maxmin_order(locs, tie)
    order = order.cpu().numpy()
    ref = S.maxmin_approx(locs, tie=tie)
    np.testing.assert_array_equal(order, ref)
    np.testing.assert_array_equal(out.cpu().numpy().reshape(locs.shape), locs[ref])


@pytest.mark.parametrize("d", [1, 2, 3, 4])
@pytest.mark.parametrize("n", [1, 2, 3, 1000, 65_537, 1 << 20])
def test_matches_the_host_ordering(d, n):
    rng = np.random.default_rng(100 * d + n % 97)
    locs = rng.random((n, d)) * np.array([2.0, 1.0, 0.25, 3.0][:d])
    check(locs, rng.random(n))


def test_clusters_repeated_ties_and_flat_axes():
    rng = np.random.default_rng(5)
    # many points per cell and repeated (also negative) ties: rank in the
    # cell, then index order among equal ties
    locs = np.column_stack([rng.integers(0, 8, 50_000) / 8.0, rng.random(50_000)])
    check(locs, rng.integers(-2, 3, 50_000).astype(float))
    # all points equal: a single cell, the order of the ties
    check(np.ones((777, 2)), rng.standard_normal(777))
    # points on a line in 3-D
    t = rng.random(4096)
    check(np.column_stack([t, np.zeros(4096), np.full(4096, -1.0)]), rng.random(4096))


def test_satellite_scaled_coordinates():
    rng = np.random.default_rng(9)
    lon, lat, _ = S.satellite_tracks(8, 16, 256, rng)
    la, lo = np.radians(lat), np.radians(lon)
    xyz = np.column_stack([np.cos(la) * np.cos(lo), np.cos(la) * np.sin(lo), np.sin(la)])
    check(xyz / S.RHO_SPACE_5DEG, rng.random(len(xyz)))

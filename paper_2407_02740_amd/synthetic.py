"""Seeded synthetic workloads shaped like the paper's data (Section 4.2).

This module is the one input source shared by the GPU library's callers and by
the test oracle.  It contains no Vecchia arithmetic: it only draws locations,
orders them, finds each observation's nearest previously ordered neighbours,
and draws a response.  The paper's datasets (Jason-3, MODIS/Terra, UCI
Elevators) are not available; these generators stand in for them with the same
shapes, sizes and structure.

Workloads (names follow the covariance model of Section 4.3, Eq. 5-6):

* ``small_exponential``  n = 2000 uniform on [0,1]^2, exact maxmin ordering,
  m = 10, exponential (sigma2, rho, tau2) = (1, 0.1, 0.01), intercept only;
  y is an exact draw of the Gaussian process (dense Cholesky of the full
  covariance, the model of Eq. 5).
* ``matern_plane``  n = 262,144 distinct points uniform on [0,1]^2 (5% exact
  duplicates drawn then removed), approximate maxmin ordering, m = 30,
  Matern nu = 3/2 (2.0, 0.05, 0.05), X = [1, x1, x2], beta = (1, -0.5, 0.3).
* ``satellite_spacetime``  64 time slices x 64 passes x 256 points along
  sinusoidal ground tracks (|lat| <= 60 deg, along-track banding), locations
  embedded in R^3 on the unit sphere plus time (Section 4.3: satellite data in
  R^3), space-time exponential (1.0, rho_s = chord of 5 deg, rho_t = 3 slices,
  0.1), m = 30, intercept only.
* ``surrogate_plane``  n = 4,194,304 uniform on [0,1]^2, approximate maxmin
  ordering, m = 30, Matern 3/2 (1.0, 0.05, 0.05), intercept only.
* ``batched_uneven``  512 independent datasets uniform on [0,1]^2, n uniform
  in [1000, 50000], m drawn from {10, 20, 30, 40}, Matern with per-dataset
  log-range ~ U[log 0.02, log 0.3], smoothness from {1/2, 3/2, 5/2} and
  nugget ratio ~ U[0.01, 0.5], variance 1, intercept only; concatenated
  arrays with per-dataset offsets.

For the large workloads the response is a random-Fourier-feature draw of
the same stationary covariance plus the nugget noise (not a Vecchia draw), so
that this module stays free of the method's arithmetic.
"""

from __future__ import annotations

import math
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

FAMILY_ISO = 0
FAMILY_SPACETIME = 1
FAMILY_ANISO = 2


# ----------------------------------------------------------------------------
# ordering
# ----------------------------------------------------------------------------
def maxmin_exact(locs: np.ndarray) -> np.ndarray:
    """Exact maxmin ordering: start at the point nearest the centroid, then
    repeatedly take the point farthest from all points taken so far."""
    n = len(locs)
    order = np.empty(n, dtype=np.int64)
    first = int(np.argmin(((locs - locs.mean(0)) ** 2).sum(1)))
    mind = ((locs - locs[first]) ** 2).sum(1)
    mind[first] = -1.0
    order[0] = first
    for k in range(1, n):
        j = int(np.argmax(mind))
        order[k] = j
        dj = ((locs - locs[j]) ** 2).sum(1)
        np.minimum(mind, dj, out=mind)
        mind[j] = -1.0
        # points already taken keep -1 (dj >= 0 never lowers them below -1)
    return order


def maxmin_approx(locs: np.ndarray, seed: int = 0, tie: np.ndarray | None = None) -> np.ndarray:
    """Approximate maxmin ordering by bit-reversed Morton codes.

    Coordinates are quantised to a 2^B grid per dimension (B chosen so a cell
    holds about one point); the interleaved cell code is bit-reversed so that
    coarse lattices come first and finer ones fill in between (coarse to
    fine); points of a cell are ranked by ``tie`` (uniform draws from
    ``seed`` unless given; equal ties by input index).
    """
    n, d = locs.shape
    rng = np.random.default_rng(seed)
    lo = locs.min(0)
    span = np.maximum(locs.max(0) - lo, 1e-300)
    B = max(1, int(math.ceil(math.log2(max(n, 2)) / d)))
    B = min(B, 60 // d)
    q = np.minimum(((locs - lo) / span * (1 << B)).astype(np.int64), (1 << B) - 1)
    code = np.zeros(n, dtype=np.int64)
    bit = 0
    # interleave from the most significant grid bit down
    for b in range(B - 1, -1, -1):
        for k in range(d):
            code |= ((q[:, k] >> b) & 1) << (B * d - 1 - bit)
            bit += 1
    # bit-reverse the B*d-bit code
    rev = np.zeros(n, dtype=np.int64)
    for b in range(B * d):
        rev |= ((code >> b) & 1) << (B * d - 1 - b)
    if tie is None:
        tie = rng.random(n)
    # several points can share a cell: a cell's k-th point comes after every
    # cell's (k-1)-th point, so each pass over the cells is coarse to fine
    by_cell = np.lexsort((tie, rev))
    sorted_rev = rev[by_cell]
    start = np.r_[0, np.flatnonzero(np.diff(sorted_rev)) + 1]
    rank_sorted = np.arange(n) - np.repeat(start, np.diff(np.r_[start, n]))
    rank = np.empty(n, dtype=np.int64)
    rank[by_cell] = rank_sorted
    return np.lexsort((tie, rev, rank))


# ----------------------------------------------------------------------------
# nearest previously ordered neighbours
# ----------------------------------------------------------------------------
def find_ordered_nn(locs: np.ndarray, m: int, workers: int = -1, log=None) -> np.ndarray:
    """NNarray[n][m+1] (int32, 0-based): row i = [i, its min(i, m) nearest
    neighbours among observations 0..i-1 by increasing distance, -1 ...]."""
    from scipy.spatial import cKDTree

    n = len(locs)
    NN = np.full((n, m + 1), -1, dtype=np.int32)
    NN[:, 0] = np.arange(n, dtype=np.int32)
    if m == 0:
        return NN
    # brute force for the first few points
    head = min(n, max(4 * (m + 1), 64))
    for i in range(1, head):
        q = min(i, m)
        dist = ((locs[:i] - locs[i]) ** 2).sum(1)
        idx = np.argsort(dist, kind="stable")[:q]
        NN[i, 1:q + 1] = idx
    # doubling blocks: a tree on points [0, b1) serves queries for [b0, b1)
    b0 = head
    while b0 < n:
        b1 = min(n, 2 * b0)
        tree = cKDTree(locs[:b1])
        rows = np.arange(b0, b1)
        k = min(b1, 3 * (m + 1))
        todo = rows
        while len(todo):
            dist, idx = tree.query(locs[todo], k=k, workers=workers)
            if k == 1:
                idx = idx[:, None]
            valid = idx < todo[:, None]
            cnt = valid.sum(1)
            ok = cnt >= m
            if ok.any():
                sel_rows = todo[ok]
                v = valid[ok]
                ii = idx[ok]
                # first m valid entries in distance order
                pos = np.cumsum(v, axis=1)
                keep = v & (pos <= m)
                NN[sel_rows, 1:] = ii[keep].reshape(-1, m)
            todo = todo[~ok]
            if k >= b1:
                break
            k = min(b1, 2 * k)
        if log:
            log(f"neighbours of observations [{b0}, {b1}) found")
        b0 = b1
    return NN


def group_cells(locs: np.ndarray, g: int, m: int, seed: int = 0):
    """Blocks of at most g nearby points and their conditioning sets, for
    grouped Vecchia.  Points are binned on a grid with about g points per
    cell (a cell with more is split into chunks of g); blocks are ordered
    coarse to fine by their centroids (the bit-reversed Morton ordering);
    block b's conditioning set is the m points before it, in the new order,
    nearest to any of its members (ties by index).

    Returns (order, block_start, cond_start, cond): order[k] is the input
    index of the k-th reordered point, block b holds reordered points
    [block_start[b], block_start[b + 1]), and cond[cond_start[b]:
    cond_start[b + 1]] (int32, indices into the reordered points, each below
    block_start[b]) is its conditioning set, nearest first."""
    from scipy.spatial import cKDTree

    n, d = locs.shape
    lo = locs.min(0)
    span = np.maximum(locs.max(0) - lo, 1e-300)
    per = max(1, int(round((n / g) ** (1.0 / d))))
    cell = np.minimum(((locs - lo) / span * per).astype(np.int64), per - 1)
    key = np.zeros(n, dtype=np.int64)
    for k in range(d):
        key = key * per + cell[:, k]
    by = np.argsort(key, kind="stable")
    ks = key[by]
    starts = np.r_[0, np.flatnonzero(np.diff(ks)) + 1, n]
    blocks = []
    for a, b in zip(starts[:-1], starts[1:]):
        for c in range(a, b, g):
            blocks.append(by[c:min(b, c + g)])
    cent = np.array([locs[bl].mean(0) for bl in blocks])
    border = maxmin_approx(cent, seed)
    order = np.concatenate([blocks[j] for j in border])
    sizes = np.array([len(blocks[j]) for j in border])
    block_start = np.r_[0, np.cumsum(sizes)].astype(np.int64)
    pts = locs[order]
    nb = len(sizes)
    member_block = np.repeat(np.arange(nb), sizes)
    bstart_of = block_start[member_block]
    cond_lists = [None] * nb
    # doubling chunks of the reordered points: a tree on [0, hi) serves the
    # blocks that start in [lo_, hi)
    lo_ = 0
    first = 0
    while first < nb:
        hi = max(2 * max(lo_, 1), int(block_start[first + 1]))
        last = int(np.searchsorted(block_start, hi, side="left")) - 1
        last = min(max(last, first), nb - 1)
        hi = int(block_start[last + 1])
        tree = cKDTree(pts[:hi])
        mem = np.arange(block_start[first], hi)
        kq = min(hi, m + g + 8)
        while True:
            dist, idx = tree.query(pts[mem], k=kq)
            if kq == 1:
                dist, idx = dist[:, None], idx[:, None]
            valid = idx < bstart_of[mem][:, None]
            need = np.minimum(m, bstart_of[mem])
            if np.all(valid.sum(1) >= need) or kq >= hi:
                break
            kq = min(hi, 2 * kq)
        for bb in range(first, last + 1):
            sl = slice(block_start[bb] - block_start[first], block_start[bb + 1] - block_start[first])
            dd, ii = dist[sl][valid[sl]], idx[sl][valid[sl]]
            if len(ii) == 0:
                cond_lists[bb] = np.zeros(0, dtype=np.int64)
                continue
            o = np.lexsort((ii, dd))
            ii = ii[o]
            _, keep = np.unique(ii, return_index=True)
            ii = ii[np.sort(keep)][:m]
            cond_lists[bb] = ii
        lo_ = hi
        first = last + 1
    cond_start = np.r_[0, np.cumsum([len(c) for c in cond_lists])].astype(np.int64)
    cond = np.concatenate(cond_lists).astype(np.int32) if nb else np.zeros(0, np.int32)
    return order, block_start, cond_start, cond


# ----------------------------------------------------------------------------
# responses
# ----------------------------------------------------------------------------
def rff_field(scaled_locs: np.ndarray, nu: float, n_features: int, rng,
              chunk: int = 1 << 16) -> np.ndarray:
    """Unit-variance draw of a stationary Matern field in already range-scaled
    coordinates by random Fourier features.  For correlation f_nu(|x|) with
    h = |x| (no sqrt(2 nu) factor) the spectral density is proportional to
    (1 + |w|^2)^-(nu + D/2), i.e. w = Z / sqrt(V), Z ~ N(0, I_D), V ~ chi2(2 nu)."""
    n, D = scaled_locs.shape
    Z = rng.standard_normal((n_features, D))
    V = rng.chisquare(2.0 * nu, size=n_features)
    W = Z / np.sqrt(V)[:, None]
    phase = rng.uniform(0.0, 2.0 * np.pi, size=n_features)
    out = np.empty(n)
    scale = math.sqrt(2.0 / n_features)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        out[a:b] = scale * np.cos(scaled_locs[a:b] @ W.T + phase).sum(1)
    return out


def _exact_gp_draw(locs, covparms, rng):
    """Exact draw of the model of Eq. 5 (exponential covariance plus nugget)."""
    sigma2, rho, tau2 = covparms
    diff = locs[:, None, :] - locs[None, :, :]
    dist = np.sqrt((diff ** 2).sum(-1))
    S = sigma2 * np.exp(-dist / rho) + sigma2 * tau2 * np.eye(len(locs))
    C = np.linalg.cholesky(S)
    return C @ rng.standard_normal(len(locs))


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------
def _pack(name, locs, NN, y, X, covparms, family, nu, nspace, m):
    return dict(name=name, locs=np.ascontiguousarray(locs, dtype=np.float64),
                NN=np.ascontiguousarray(NN, dtype=np.int32),
                y=np.ascontiguousarray(y, dtype=np.float64),
                X=np.ascontiguousarray(X, dtype=np.float64),
                covparms=np.asarray(covparms, dtype=np.float64), family=family, nu=float(nu),
                nspace=int(nspace), m=int(m), n=len(y), p=X.shape[1], d=locs.shape[1])


def small_exponential(seed: int = 1, n: int = 2000, m: int = 10) -> dict:
    rng = np.random.default_rng(seed)
    locs = rng.random((n, 2))
    locs = locs[maxmin_exact(locs)]
    NN = find_ordered_nn(locs, m)
    covparms = (1.0, 0.1, 0.01)
    y = _exact_gp_draw(locs, covparms, rng)
    X = np.ones((n, 1))
    return _pack("small_exponential", locs, NN, y, X, covparms, FAMILY_ISO, 0.5, 0, m)


def matern_plane(seed: int = 2, n: int = 262_144, m: int = 30, n_features: int = 512) -> dict:
    rng = np.random.default_rng(seed)
    base = rng.random((n, 2))
    dup = base[rng.integers(0, n, size=int(0.05 * n))]
    pts = np.concatenate([base, dup])
    _, first = np.unique(pts, axis=0, return_index=True)
    pts = pts[np.sort(first)]
    while len(pts) < n:
        extra = rng.random((n - len(pts), 2))
        pts = np.concatenate([pts, extra])
        _, first = np.unique(pts, axis=0, return_index=True)
        pts = pts[np.sort(first)]
    locs = pts[:n]
    order = maxmin_exact(locs) if n <= 20_000 else maxmin_approx(locs, seed)
    locs = locs[order]
    NN = find_ordered_nn(locs, m)
    covparms = (2.0, 0.05, 0.05)
    nu = 1.5
    X = np.column_stack([np.ones(n), locs[:, 0], locs[:, 1]])
    beta = np.array([1.0, -0.5, 0.3])
    f = rff_field(locs / covparms[1], nu, n_features, rng)
    y = X @ beta + math.sqrt(covparms[0]) * f + math.sqrt(covparms[0] * covparms[2]) * \
        rng.standard_normal(n)
    return _pack("matern_plane", locs, NN, y, X, covparms, FAMILY_ISO, nu, 0, m)


RHO_SPACE_5DEG = 2.0 * math.sin(math.radians(2.5))  # chord length of a 5 degree arc


def satellite_tracks(slices: int, passes: int, per_pass: int, rng):
    """lon/lat/time of points along sinusoidal ground tracks.

    Each pass covers half an orbit: lat = 60 deg * sin(phi), lon = lon0 + phi
    (degrees, wrapped to [-180, 180)), phi uniform on [0, pi), alternately
    ascending and descending; t = slice index + a uniform offset that
    increases along the pass."""
    lon = np.empty((slices, passes, per_pass))
    lat = np.empty_like(lon)
    t = np.empty_like(lon)
    for s in range(slices):
        for k in range(passes):
            phi = np.sort(rng.uniform(0.0, np.pi, per_pass))
            if k % 2:
                phi = phi[::-1]
            lon0 = rng.uniform(-180.0, 180.0)
            lat[s, k] = 60.0 * np.sin(phi) * (1 if k % 2 == 0 else -1)
            lon[s, k] = (lon0 + np.degrees(phi) + 180.0) % 360.0 - 180.0
            t[s, k] = s + np.sort(rng.uniform(0.0, 1.0, per_pass))
    return lon.ravel(), lat.ravel(), t.ravel()


def satellite_spacetime(seed: int = 3, slices: int = 64, passes: int = 64, per_pass: int = 256,
                        m: int = 30, n_features: int = 512) -> dict:
    rng = np.random.default_rng(seed)
    lon, lat, t = satellite_tracks(slices, passes, per_pass, rng)
    la, lo = np.radians(lat), np.radians(lon)
    xyz = np.column_stack([np.cos(la) * np.cos(lo), np.cos(la) * np.sin(lo), np.sin(la)])
    locs = np.column_stack([xyz, t])
    covparms = (1.0, RHO_SPACE_5DEG, 3.0, 0.1)
    scaled = np.column_stack([xyz / covparms[1], t / covparms[2]])
    n = len(locs)
    order = maxmin_exact(scaled) if n <= 20_000 else maxmin_approx(scaled, seed)
    locs, scaled = locs[order], scaled[order]
    NN = find_ordered_nn(scaled, m)
    nu = 0.5
    f = rff_field(scaled, nu, n_features, rng)
    X = np.ones((n, 1))
    y = 0.5 + math.sqrt(covparms[0]) * f + math.sqrt(covparms[0] * covparms[3]) * \
        rng.standard_normal(n)
    return _pack("satellite_spacetime", locs, NN, y, X, covparms, FAMILY_SPACETIME, nu, 3, m)


def attributes_18d(seed: int = 6, n: int = 14_939, d: int = 18, m: int = 30,
                   n_features: int = 1024) -> dict:
    """Regression on attribute vectors, the shape of the 18-attribute UCI
    data of Section 4.2 (about 15,000 training rows per fold): standardised
    attributes of mixed marginals (Gaussian, uniform, skewed, few-valued) used
    as locations, an exponential covariance with one range per attribute
    (Eq. 6), ranges log-uniform on [1, 20] so that some attributes matter far
    more than others, nugget ratio 0.1, constant mean.  Random ordering (as in
    the timing study of Section 4); neighbours by distance in range-scaled
    coordinates."""
    rng = np.random.default_rng(seed)
    cols = []
    for k in range(d):
        kind = k % 4
        if kind == 0:
            c = rng.standard_normal(n)
        elif kind == 1:
            c = rng.random(n)
        elif kind == 2:
            c = rng.lognormal(0.0, 0.75, n)
        else:
            c = rng.integers(0, 6, n) + 0.05 * rng.standard_normal(n)
        cols.append((c - c.mean()) / c.std())
    locs = np.column_stack(cols)
    rho = np.exp(rng.uniform(math.log(1.0), math.log(20.0), d))
    covparms = np.concatenate([[1.0], rho, [0.1]])
    locs = locs[rng.permutation(n)]
    scaled = locs / rho
    NN = find_ordered_nn(scaled, m)
    f = rff_field(scaled, 0.5, n_features, rng)
    y = 0.3 + f + math.sqrt(covparms[-1]) * rng.standard_normal(n)
    X = np.ones((n, 1))
    return _pack("attributes_18d", locs, NN, y, X, covparms, FAMILY_ANISO, 0.5, 0, m)


def _one_dataset(args):
    seed_seq, n_min, n_max, ms, n_features, rho_range, tau2_range = args
    rng = np.random.default_rng(seed_seq)
    n = int(rng.integers(n_min, n_max + 1))
    m = int(rng.choice(ms))
    rho = math.exp(rng.uniform(math.log(rho_range[0]), math.log(rho_range[1])))
    nu = float(rng.choice([0.5, 1.5, 2.5]))
    tau2 = float(rng.uniform(*tau2_range))
    locs = rng.random((n, 2))
    locs = locs[maxmin_approx(locs, int(rng.integers(1 << 30)))]
    NN = find_ordered_nn(locs, m, workers=1)
    f = rff_field(locs / rho, nu, n_features, rng)
    y = 0.2 + f + math.sqrt(tau2) * rng.standard_normal(n)
    return locs, NN, y, m, nu, (1.0, rho, tau2)


def batched_uneven(seed: int = 4, nsets: int = 512, n_min: int = 1000, n_max: int = 50_000,
                   ms=(10, 20, 30, 40), n_features: int = 256, workers: int | None = None,
                   rho_range=(0.02, 0.3), tau2_range=(0.01, 0.5)) -> dict:
    """Independent 2-D datasets of uneven n and m, concatenated.  Dataset b
    draws from its own child seed, so the result does not depend on the
    number of worker processes."""
    children = np.random.SeedSequence(seed).spawn(nsets)
    jobs = [(c, n_min, n_max, tuple(ms), n_features, tuple(rho_range), tuple(tau2_range))
            for c in children]
    workers = workers or min(16, os.cpu_count() or 1)
    if workers > 1 and nsets > 1:
        with ProcessPoolExecutor(workers) as ex:
            parts = list(ex.map(_one_dataset, jobs, chunksize=4))
    else:
        parts = [_one_dataset(j) for j in jobs]
    n = np.array([len(p[2]) for p in parts], dtype=np.int64)
    m = np.array([p[3] for p in parts], dtype=np.int64)
    obs_offset = np.concatenate([[0], np.cumsum(n)[:-1]])
    nn_sizes = n * (m + 1)
    nn_offset = np.concatenate([[0], np.cumsum(nn_sizes)[:-1]])
    locs = np.concatenate([p[0] for p in parts])
    NN = np.concatenate([p[1].reshape(-1) for p in parts]).astype(np.int32)
    y = np.concatenate([p[2] for p in parts])
    return dict(name="batched_uneven", locs=np.ascontiguousarray(locs), NN=NN, y=y,
                X=np.ones((len(y), 1)), n=n, m=m, obs_offset=obs_offset, nn_offset=nn_offset,
                nu=np.array([p[4] for p in parts]), covparms=np.array([p[5] for p in parts]),
                family=FAMILY_ISO, nspace=0, d=2, p=1, nsets=nsets)


def batch_member(w: dict, b: int) -> dict:
    """Dataset b of a batched workload as a single problem."""
    a, n, m = int(w["obs_offset"][b]), int(w["n"][b]), int(w["m"][b])
    o = int(w["nn_offset"][b])
    NN = w["NN"][o:o + n * (m + 1)].reshape(n, m + 1)
    return _pack(f"{w['name']}[{b}]", w["locs"][a:a + n], NN, w["y"][a:a + n], w["X"][a:a + n],
                 tuple(w["covparms"][b]), w["family"], float(w["nu"][b]), w["nspace"], m)


def surrogate_plane(seed: int = 5, n: int = 4_194_304, m: int = 30, n_features: int = 512,
                    log=None) -> dict:
    """The surrogate's evaluation problem: n uniform points on [0,1]^2,
    approximate maxmin ordering, m = 30, Matern 3/2 (1.0, 0.05, 0.05),
    intercept only."""
    rng = np.random.default_rng(seed)
    locs = rng.random((n, 2))
    order = maxmin_exact(locs) if n <= 20_000 else maxmin_approx(locs, seed)
    locs = locs[order]
    NN = find_ordered_nn(locs, m, log=log)
    covparms = (1.0, 0.05, 0.05)
    nu = 1.5
    f = rff_field(locs / covparms[1], nu, n_features, rng)
    y = 0.3 + math.sqrt(covparms[0]) * f + math.sqrt(covparms[0] * covparms[2]) * \
        rng.standard_normal(n)
    return _pack("surrogate_plane", locs, NN, y, np.ones((n, 1)), covparms, FAMILY_ISO, nu, 0, m)


def nn_among(locs_obs: np.ndarray, locs_pred: np.ndarray, m: int) -> np.ndarray:
    """Prediction rows of an NNarray: for prediction point j (appended after
    the n_obs observations), [n_obs + j, its m nearest observed points by
    increasing distance] (int32 [n_pred][m + 1])."""
    from scipy.spatial import cKDTree

    n_obs = len(locs_obs)
    _, idx = cKDTree(locs_obs).query(locs_pred, k=m, workers=-1)
    idx = np.asarray(idx).reshape(len(locs_pred), m)
    out = np.empty((len(locs_pred), m + 1), dtype=np.int32)
    out[:, 0] = n_obs + np.arange(len(locs_pred))
    out[:, 1:] = idx
    return out

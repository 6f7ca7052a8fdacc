"""The allocation-free entry point against the one that takes a workspace.

vecchia_loglik_grad_info_noalloc keeps its partial sums in the library's
per-device scratch array instead of a caller workspace and runs the same
kernels on the same grid, so its raw sums and outputs must equal those of
vecchia_loglik_grad_info bit for bit.  Two calls in a row, the second on a
smaller problem of another family, show that the scratch contents left by
the first call do not leak into the second; the first result is also checked
against the oracle at the parity tolerances.
"""

import ctypes

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


def _plane(n, m, seed):
    rng = np.random.default_rng(seed)
    locs = rng.random((n, 2))
    locs = locs[S.maxmin_exact(locs)]
    NN = S.find_ordered_nn(locs, m)
    y = rng.standard_normal(n) + 0.3 * np.sin(7 * locs[:, 0])
    X = np.column_stack([np.ones(n), locs[:, 0]])
    return dict(locs=locs, NN=NN, y=y, X=X, family=V.FAMILY_ISO, nu=1.5, nspace=0, n=n, m=m, p=2,
                covparms=np.array((1.3, 0.12, 0.05)))


def _both(w):
    ev = V.Vecchia(w["locs"], w["NN"], w["y"], w["X"], w["family"], w["nu"], w["nspace"])
    ev.loglik_grad_info(w["covparms"])
    torch.cuda.synchronize()
    raw_ws, out_ws = ev.raw.clone(), ev.out.clone()
    ev.raw.fill_(float("nan"))
    ev.out.fill_(float("nan"))
    ev.loglik_grad_info_noalloc(w["covparms"])
    torch.cuda.synchronize()
    return ev, raw_ws, out_ws, ev.raw.clone(), ev.out.clone()


def test_noalloc_equals_workspace_entry_point_twice():
    big = S.satellite_spacetime(slices=4, passes=8, per_pass=128, m=30)
    small = _plane(700, 10, seed=11)
    for tag, w in (("space-time n=4096 m=30", big), ("Matern plane n=700 m=10", small)):
        _say(f"case {tag}")
        ev, raw_ws, out_ws, raw_na, out_na = _both(w)
        assert torch.equal(raw_ws, raw_na), tag
        assert torch.equal(out_ws, out_na), tag
        if w is big:
            got = V.unpack_out(out_na, w["p"], ev.P)
            ref = oracle.loglik_grad_info(w["locs"], w["NN"], w["y"], w["X"], w["covparms"],
                                          w["family"], w["nu"], w["nspace"])
            assert abs(got["loglik"] - ref["loglik"]) <= 1e-10 * abs(ref["loglik"])
            sd = np.sqrt(np.diag(ref["info"]))
            assert np.all(np.abs(got["grad"] - ref["grad"])
                          <= 1e-8 * np.maximum(np.abs(ref["grad"]), sd))
            assert np.all(np.abs(got["info"] - ref["info"])
                          <= 1e-8 * np.maximum(np.abs(ref["info"]), np.outer(sd, sd)))


def test_noalloc_rejects_problems_beyond_the_scratch_array():
    # one range per coordinate at d = 32: nraw = 1,646 doubles per workgroup,
    # far beyond 2 MiB of partial sums for a full grid
    L = V.lib()
    pb = V.Problem(n=100000, m=30, d=32, p=3, family=V.FAMILY_ANISO, smoothness=0.5, nspace=0)
    assert L.vec_workspace_bytes(ctypes.byref(pb), 0, pb.n) > (2 << 20)
    fake = ctypes.c_void_p(256)
    rc = L.vecchia_loglik_grad_info_noalloc(ctypes.byref(pb), fake, fake, fake, fake, fake, fake,
                                            fake, fake, None)
    assert rc == V.VEC_EWORKSPACE

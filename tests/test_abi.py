"""The C ABI library loads on the host and exports every declared symbol.

No GPU work happens here: only entry points that validate arguments on the
host before touching the device are called.
"""

import ctypes
import os
import re

import pytest

from paper_2407_02740_amd import vecchia as V

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("vecchia.h", "vecchia_surrogate.h")]

pytestmark = pytest.mark.skipif(not os.path.exists(V.LIB_PATH), reason="libvecchia.so not built")


def declared_symbols():
    text = "".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vec(?:chia)?_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L = ctypes.CDLL(V.LIB_PATH)
    syms = declared_symbols()
    assert len(syms) >= 30
    for s in syms:
        assert hasattr(L, s), s


def test_problem_sizes_and_validation_on_host():
    L = V.lib()
    pb = V.Problem(n=1000, m=30, d=4, p=1, family=V.FAMILY_SPACETIME, smoothness=0.5, nspace=3)
    assert L.vec_nparms(ctypes.byref(pb)) == 4
    assert L.vec_nraw(ctypes.byref(pb)) == 36
    assert L.vec_nout(ctypes.byref(pb)) == 1 + 4 + 16 + 1 + 1
    pb2 = V.Problem(n=1000, m=30, d=2, p=3, family=V.FAMILY_ISO, smoothness=1.5, nspace=0)
    assert L.vec_nraw(ctypes.byref(pb2)) == 65
    assert L.vec_max_m() == 60
    # beyond the fused kernel's sizes the sums still accept m <= 63
    pb3 = V.Problem(n=1000, m=60, d=2, p=1, family=V.FAMILY_ISO, smoothness=0.5, nspace=0)
    assert L.vec_nparms(ctypes.byref(pb3)) == 3
    bad = [
        dict(n=0), dict(m=64), dict(d=5), dict(p=0), dict(p=4), dict(family=7),
        dict(smoothness=1.0), dict(nspace=0), dict(nspace=4), dict(reserved=1),
    ]
    for change in bad:
        args = dict(n=1000, m=30, d=4, p=1, family=V.FAMILY_SPACETIME, smoothness=0.5, nspace=3)
        args.update(change)
        pbx = V.Problem(**{k: v for k, v in args.items() if k != "reserved"})
        pbx.reserved = args.get("reserved", 0)
        assert L.vec_nparms(ctypes.byref(pbx)) == V.VEC_EINVAL, change
    # one range per coordinate: P = d + 2 up to d = 32, m up to 63
    pa = V.Problem(n=15000, m=30, d=18, p=1, family=V.FAMILY_ANISO, smoothness=0.5, nspace=0)
    assert L.vec_nparms(ctypes.byref(pa)) == 20
    assert L.vec_nraw(ctypes.byref(pa)) == 2 + 1 + 1 + 20 * 4 + 400
    for change in [dict(d=33), dict(m=64), dict(p=4), dict(smoothness=2.0), dict(d=0)]:
        args = dict(n=15000, m=30, d=18, p=1, family=V.FAMILY_ANISO, smoothness=0.5, nspace=0)
        args.update(change)
        assert L.vec_nparms(ctypes.byref(V.Problem(**args))) == V.VEC_EINVAL, change
    for ok in [dict(d=32, m=63, p=3), dict(d=1, m=0)]:
        args = dict(n=15000, m=30, d=18, p=1, family=V.FAMILY_ANISO, smoothness=1.5, nspace=0)
        args.update(ok)
        assert L.vec_nparms(ctypes.byref(V.Problem(**args))) == args["d"] + 2, ok
    # null pointers and bad ranges are rejected before anything is enqueued
    null = None
    rc = L.vec_raw_sums(ctypes.byref(pb), null, null, null, null, null, 0, 1000, null, null, 0,
                        null, null)
    assert rc == V.VEC_EINVAL
    fake = ctypes.c_void_p(8)
    rc = L.vec_raw_sums(ctypes.byref(pb), fake, fake, fake, fake, fake, 10, 5, fake, fake, 0, fake,
                        null)
    assert rc == V.VEC_EINVAL
    rc = L.vec_raw_sums(ctypes.byref(pb), fake, fake, fake, fake, fake, 0, 1001, fake, fake, 0,
                        fake, null)
    assert rc == V.VEC_EINVAL


def test_status_decoding():
    L = V.lib()

    def code(a, b):
        return L.vec_status_code((ctypes.c_int32 * 2)(a, b))

    assert code(0, 2 ** 31 - 1) == V.VEC_OK
    assert code(1, 5) == V.VEC_ENOTPD
    assert code(2, 5) == V.VEC_EBADNN
    assert code(3, 5) == V.VEC_EBADNN
    assert code(4, 5) == V.VEC_ENONFINITE


def test_batch_plan_validation_on_host():
    """Invalid batches, descriptors and schedules are rejected before any
    device call (no GPU needed)."""
    L = V._batch_lib()
    assert L.vec_batch_plan_bytes(0) == 0 and L.vec_batch_plan_bytes(70000) == 0
    assert L.vec_batch_plan_bytes(512) > 512 * 8 * 8
    fake = ctypes.c_void_p(256)
    big = 1 << 40

    def plan(bt_kw=None, sets=None, sched=None):
        bt = V.Batch(nsets=2, d=2, p=1, family=V.FAMILY_ISO, nspace=0, reserved=0, n_total=300,
                     nn_total=300 * 41)
        for k, v in (bt_kw or {}).items():
            setattr(bt, k, v)
        arr = (V.Dataset * 2)()
        base = [dict(obs_offset=0, nn_offset=0, n=100, m=10, reserved=0, smoothness=0.5),
                dict(obs_offset=100, nn_offset=1100, n=200, m=40, reserved=0, smoothness=2.5)]
        for b in range(2):
            kw = {**base[b], **((sets or {}).get(b, {}))}
            arr[b] = V.Dataset(**kw)
        pl = V.Plan()
        return L.vec_batch_make_plan(ctypes.byref(bt), arr,
                                     ctypes.byref(sched) if sched is not None else None,
                                     ctypes.byref(pl), fake, big, None)

    bad = [
        dict(bt_kw=dict(nsets=0)), dict(bt_kw=dict(d=5)), dict(bt_kw=dict(p=0)),
        dict(bt_kw=dict(family=3)), dict(bt_kw=dict(family=V.FAMILY_ANISO)),
        dict(bt_kw=dict(reserved=1)), dict(bt_kw=dict(n_total=299)),
        dict(bt_kw=dict(nn_total=1100 + 200 * 41 - 1)),
        dict(sets={0: dict(n=0)}), dict(sets={0: dict(m=-1)}), dict(sets={1: dict(m=41)}),
        dict(sets={0: dict(smoothness=1.0)}), dict(sets={0: dict(reserved=2)}),
        dict(sets={1: dict(obs_offset=101)}), dict(sets={0: dict(obs_offset=-1)}),
        dict(sets={1: dict(nn_offset=300 * 41 - 200 * 41 + 1)}), dict(sets={0: dict(nn_offset=-5)}),
        dict(sched=V.schedule(tile=-1)), dict(sched=V.schedule(tile=(1 << 21))),
        dict(sched=V.schedule(blocks_per_cu=-2)),
    ]
    for case in bad:
        assert plan(**case) == V.VEC_EINVAL, case
    # too small a plan buffer
    bt = V.Batch(nsets=2, d=2, p=1, family=V.FAMILY_ISO, nspace=0, reserved=0, n_total=300,
                 nn_total=300 * 41)
    arr = (V.Dataset * 2)()
    pl = V.Plan()
    assert L.vec_batch_make_plan(ctypes.byref(bt), arr, None, ctypes.byref(pl), fake, 16,
                                 None) == V.VEC_EWORKSPACE
    assert L.vec_batch_status_clear(None, 2, None) == V.VEC_EINVAL

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
HEADER = os.path.join(ROOT, "include", "vecchia.h")

pytestmark = pytest.mark.skipif(not os.path.exists(V.LIB_PATH), reason="libvecchia.so not built")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vec(?:chia)?_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L = ctypes.CDLL(V.LIB_PATH)
    syms = declared_symbols()
    assert len(syms) >= 12
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
    assert L.vec_max_m() >= 30
    bad = [
        dict(n=0), dict(m=L.vec_max_m() + 1), dict(d=5), dict(p=0), dict(p=4), dict(family=7),
        dict(smoothness=1.0), dict(nspace=0), dict(nspace=4), dict(reserved=1),
    ]
    for change in bad:
        args = dict(n=1000, m=30, d=4, p=1, family=V.FAMILY_SPACETIME, smoothness=0.5, nspace=3)
        args.update(change)
        pbx = V.Problem(**{k: v for k, v in args.items() if k != "reserved"})
        pbx.reserved = args.get("reserved", 0)
        assert L.vec_nparms(ctypes.byref(pbx)) == V.VEC_EINVAL, change
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

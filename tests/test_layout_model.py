"""Host model of the fused kernel's LDS copy of the factor (no GPU).

Every lane of a 16-lane group stores the row of the unit-lower factor it
owns at Lp[r (r - 1) / 2 + c] for every column c of its slot, whatever c is,
slot by slot and column by column in decreasing order; entries past the
diagonal spill into the following rows and must be overwritten later by the
entry that belongs there.  The model replays that store sequence for every
instantiated size with the adversarial rule that, when two lanes of one store
hit the same address, the wrong one wins, and checks that every entry of the
strict lower triangle ends up in place.  It mirrors the kernel's row-to-lane
map (slot s holds row 16 s + l for even s, 16 s + 15 - l for odd s) and its
row bases (row 0 and rows >= K write a sink).
"""

import pytest


def row_of(s, l):
    return 16 * s + (15 - l if s & 1 else l)


@pytest.mark.parametrize("K", [11, 21, 31])
def test_factor_copy_store_order_leaves_every_entry_in_place(K):
    NS = (K + 15) // 16
    LPN = K * (K - 1) // 2
    length = [min(16 * (s + 1), K) for s in range(NS)]
    sink = LPN + 1
    size = LPN + 1 + K
    lp = [None] * size
    for s in range(NS):
        for c in reversed(range(length[s])):
            writes = {}
            for l in range(16):
                r = row_of(s, l)
                base = r * (r - 1) // 2 if 1 <= r < K else sink
                addr = base + c
                assert 0 <= addr < size
                val = ("L", r, c) if c < r < K else ("garbage", r, c)
                writes.setdefault(addr, []).append(val)
            for addr, vals in writes.items():
                # a valid entry loses to garbage whenever two lanes collide
                garbage = [v for v in vals if v[0] == "garbage"]
                lp[addr] = garbage[0] if garbage else vals[0]
    for r in range(1, K):
        for c in range(r):
            assert lp[r * (r - 1) // 2 + c] == ("L", r, c), (K, r, c, lp[r * (r - 1) // 2 + c])

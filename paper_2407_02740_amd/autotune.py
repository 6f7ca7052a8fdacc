"""Schedule autotuner for the batched persistent launches.

Each size class (neighbourhood size m + 1 <= 11, 21, 31, 41) runs as its own
persistent launch, so its schedule can be chosen on its own: for every class
present in the batch, the class's datasets alone are evaluated under each
candidate (observations per tile, workgroups per CU) and the fastest
candidate, by the median of a few timed runs, is kept.  The neighbourhood
itself is always processed by one 16-lane DPP row of a wavefront (four per
wave); the candidates change how the observations are cut into work items
and how many persistent workgroups share them.

Host logic only: every evaluation runs in the library's kernels.
"""

from __future__ import annotations

import statistics

import torch

from . import vecchia as V

DEFAULT_TILES = (4, 8, 16, 32, 64, 128, 256)
DEFAULT_BLOCKS = (0, 2)


def _time_eval(vb: V.VecchiaBatch, cp: torch.Tensor, reps: int) -> float:
    vb.raw_sums(cp, check=False)  # warm-up (also loads the code object)
    times = []
    stream = torch.cuda.current_stream()
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        vb.raw_sums(cp, check=False)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return statistics.median(times)


def tune_batch(vb: V.VecchiaBatch, covparms, tiles=DEFAULT_TILES, blocks=DEFAULT_BLOCKS,
               reps: int = 3, log=None):
    """Pick a schedule for the batch `vb` at parameters `covparms`
    ([nsets][P]).  Returns (schedule, table) where table[c] lists
    (tile, blocks_per_cu, ms) for every candidate of class c; `vb` is left
    with a plan made from the chosen schedule."""
    cp = vb.covparms(covparms) if not (isinstance(covparms, torch.Tensor) and covparms.is_cuda) \
        else covparms
    classes = [min(c for c, K in enumerate(V.CLASS_K) if m + 1 <= K) for m in
               (s.m for s in vb.sets)]
    best_tile = [0] * V.NUM_CLASSES
    best_blocks = [0] * V.NUM_CLASSES
    table = {}
    for c in range(V.NUM_CLASSES):
        members = [b for b, k in enumerate(classes) if k == c]
        if not members:
            continue
        sub = V.VecchiaBatch(vb.locs, vb.NN, vb.y, vb.X,
                             [vb.sets[b].obs_offset for b in members],
                             [vb.sets[b].nn_offset for b in members],
                             [vb.sets[b].n for b in members], [vb.sets[b].m for b in members],
                             [vb.sets[b].smoothness for b in members], vb.bt.family,
                             vb.bt.nspace)
        sub_cp = cp[members].contiguous()
        rows = []
        for t in tiles:
            for bl in blocks:
                sub.make_plan(V.schedule(tile=t, blocks_per_cu=bl))
                ms = _time_eval(sub, sub_cp, reps)
                rows.append((t, bl, ms))
                if log:
                    log(f"class K={V.CLASS_K[c]} ({len(members)} datasets): tile {t}, "
                        f"blocks/CU {bl or 'resident'}: {ms:.3f} ms")
        sub.check_status("autotune")
        t, bl, _ = min(rows, key=lambda r: r[2])
        best_tile[c], best_blocks[c] = t, bl
        table[c] = rows
    sched = V.schedule(tile=best_tile, blocks_per_cu=best_blocks)
    vb.make_plan(sched)
    return sched, table

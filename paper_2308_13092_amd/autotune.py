"""Launch autotuner for a live context.

Picks the fused particle kernel's block size, the number of persistent blocks
per compute unit, the cell-sort interval and whether steps replay a captured
HIP graph or launch plainly, by timing whole steps of the context's own
discharges on the device.  None of these settings changes a
result: every particle's update depends only on its own state, the field and
its Philox stream, the deposit is an exact integer sum, and the sort only
reorders storage.  The steps taken while tuning are ordinary steps of the
simulation (they advance k), so callers tune during their warm-up.
"""
from __future__ import annotations

import itertools
import sys
import time

BLOCKS = (256, 512, 1024)
BLOCKS_PER_CU = (0, 1, 2, 3, 4)
SORT_INTERVALS = (10, 20, 40)
GRAPHS = (0, 1)


def _time_steps(ctx, n):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(n)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / n


def autotune(ctx, steps=40, blocks=BLOCKS, blocks_per_cu=BLOCKS_PER_CU,
             sort_intervals=SORT_INTERVALS, graphs=GRAPHS, verbose=False):
    """Time each setting over ``steps`` steps (a multiple of every sort
    interval, after a one-interval settle) and keep the fastest.  Returns the
    chosen tuning and the table of (setting, seconds per step)."""
    base = ctx.tuning()
    G0 = base["use_graph"]
    table = []
    # Launch shape first, at the context's own sort interval.
    S0 = base["sort_interval"] or 20
    for block, bpc in itertools.product(blocks, blocks_per_cu):
        ctx.set_tuning(block=block, blocks_per_cu=bpc, sort_interval=S0, use_graph=G0)
        ctx.step(S0)                      # settle (and graph capture)
        sec = _time_steps(ctx, _round_up(steps, S0))
        table.append((dict(block=block, blocks_per_cu=bpc, sort_interval=S0), sec))
        if verbose:
            print(f"[autotune] block {block} bpc {bpc}: {sec * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
    best = min(table, key=lambda r: r[1])[0]
    # Then the sort interval at that launch shape.
    sort_table = []
    for S in sort_intervals:
        ctx.set_tuning(block=best["block"], blocks_per_cu=best["blocks_per_cu"], sort_interval=S,
                       use_graph=G0)
        ctx.step(S)
        sec = _time_steps(ctx, _round_up(max(steps, 2 * S), S))
        sort_table.append((dict(best, sort_interval=S), sec))
        if verbose:
            print(f"[autotune] sort every {S}: {sec * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
    best = min(sort_table, key=lambda r: r[1])[0]
    # Last, graph replay or plain launches at that setting.
    graph_table = []
    for g in graphs:
        ctx.set_tuning(use_graph=g, **best)
        ctx.step(best["sort_interval"] or S0)
        sec = _time_steps(ctx, _round_up(steps, best["sort_interval"] or S0))
        graph_table.append((dict(best, use_graph=g), sec))
        if verbose:
            print(f"[autotune] use_graph {g}: {sec * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
    chosen = min(graph_table, key=lambda r: r[1])[0]
    ctx.set_tuning(**chosen)
    return chosen, table + sort_table + graph_table


def _round_up(n, m):
    return ((n + m - 1) // m) * m

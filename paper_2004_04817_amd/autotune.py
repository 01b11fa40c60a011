"""Autotuner of the batched launch layout (tile shapes).

Times the batched selection of a set of contexts under each candidate
layout -- targets per lane in the group sweeps, 16-row chunks per factor
wave -- on the device it will run on, and returns the fastest.  Every
candidate computes the same selection (the factor's sums do not depend on
the layout; the sweep layout changes only the summation order of the group
errors), so tuning never changes a result beyond rounding.
"""
from __future__ import annotations

import time

from . import Batch

CANDIDATES = ((0, 0), (1, 1), (1, 4), (2, 1), (2, 4), (4, 1), (4, 4))


def tune_batch(ctxs, candidates=CANDIDATES, repeats: int = 2, stream=None):
    """Return ((sweep_tpl, factor_rpw), {candidate: seconds}) for the contexts' batched selection."""
    import torch
    times = {}
    with Batch(ctxs[0].device, stream) as b:
        for cand in candidates:
            b.set_layout(*cand)
            best = float("inf")
            for _ in range(repeats):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                b.select(ctxs)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
            times[cand] = best
    return min(times, key=times.get), times

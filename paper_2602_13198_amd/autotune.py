"""Launch-parameter autotuner for the transport launches.

Results never depend on the tuning (photon histories are keyed by their
random streams), so the tuner only compares time: for each candidate
(waves per SIMD of the compiled tracker variant, idle-lane refill threshold,
instances per shared launch) it runs the caller's step once untimed and
`repeats` times timed, and keeps the one with the shortest wall time; the
summed tracking-kernel event time is logged beside it.
"""
from __future__ import annotations

import itertools
import time

DEFAULT_CANDIDATES = (list(itertools.product((2, 3, 4), (8, 16, 32), (1, 64)))
                      + [(2, 12, 64), (2, 24, 64)])


def autotune(ctx, step, candidates=None, repeats: int = 1, log=None):
    """ctx: gm.Context; step(seed) runs one full make/track/read step.
    Returns (best (waves, refill, batch), list of (waves, refill, batch,
    track_ms, wall_ms))."""
    import torch
    table = []
    seed = 900000
    for waves, refill, batch in (candidates or DEFAULT_CANDIDATES):
        ctx.set_tuning(waves, refill)
        ctx.set_batch(batch)
        step(seed)
        seed += 1
        torch.cuda.synchronize()
        ctx.set_timing(True)
        t0 = time.perf_counter()
        for _ in range(repeats):
            step(seed)
            seed += 1
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / repeats
        ms, _ = ctx.read_timing()
        ctx.set_timing(False)
        table.append((waves, refill, batch, ms / repeats, wall))
        if log:
            log("tune waves=%d refill=%d batch=%d: track %.2f ms, step %.2f ms"
                % (waves, refill, batch, ms / repeats, wall))
    best = min(table, key=lambda r: r[4])
    ctx.set_tuning(best[0], best[1])
    ctx.set_batch(best[2])
    return (best[0], best[1], best[2]), table

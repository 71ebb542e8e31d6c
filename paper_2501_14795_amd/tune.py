"""Autotuner for the batched mode: times candidate launch configurations on
graph replays of the actual batch and keeps the fastest.  A candidate is
(tile size, LDS current replicas, sort cadence, particles per lane, sort): the
tile size sets the work per workgroup and the halo overhead, the sort cadence
how many pushes run between two sorts, the particles per lane how many
64-particle chunks a wavefront of the push carries side by side (more chunks:
more independent work to cover latencies; fewer: fewer registers, more
resident wavefronts), and the sort is the in-place one (moves only the
particles that left their section) or the motion-class one (moves every
particle once, out of place; for plasmas where most particles change tile).
The particle arrays must be grouped by tile for each candidate tile size, so
the caller supplies a function that builds the members' initial states for a
given tile size."""
from __future__ import annotations

import time
from typing import Callable, Dict, Sequence, Tuple

# (tile, replicas, sort_every, particles per lane, motion-class sort); a
# 4-tuple means the in-place sort
Candidate = Tuple

DEFAULT_CANDIDATES: Tuple[Candidate, ...] = (
    (8, 1, 1, 2, False), (8, 1, 2, 2, False), (8, 1, 1, 1, False),
    (16, 1, 1, 2, False), (16, 2, 1, 2, False), (16, 1, 2, 2, False), (16, 1, 4, 2, False),
    (16, 1, 1, 1, False), (16, 1, 1, 4, False), (16, 1, 2, 1, False), (16, 1, 2, 4, False),
    (32, 1, 1, 2, False), (32, 1, 2, 2, False), (32, 1, 1, 1, False), (32, 1, 1, 4, False),
    (8, 1, 1, 2, True), (16, 1, 1, 2, True), (16, 1, 2, 2, True))


def time_batch(batch, steps: int) -> float:
    """Seconds per step of `batch` (graph-replayed if captured), over whole
    sort-cadence cycles after one cycle of warm-up."""
    k = max(1, int(getattr(batch, "sort_every", 1)))
    steps = -(-steps // k) * k
    batch.step(k)
    batch.stream.synchronize()
    t0 = time.perf_counter()
    batch.step(steps)
    batch.sync()   # the last sort's hole fill, which the next push would do
    batch.stream.synchronize()
    return (time.perf_counter() - t0) / steps


def autotune_batch(build_members: Callable[[int], Sequence[dict]],
                   candidates: Sequence[Candidate] = DEFAULT_CANDIDATES,
                   steps: int = 4, j_float: bool = False) -> Tuple[Candidate, Dict[Candidate, float]]:
    """Returns (best candidate, {candidate: seconds per step}); candidates the
    library refuses (LDS budget, a cadence the tile cannot take, particles per
    lane outside the default current) or whose grids are not whole tiles are
    skipped."""
    from .sim import Batch
    from . import _lib
    timings: Dict[Candidate, float] = {}
    for cand in candidates:
        tile, reps, every, ppl = cand[:4]
        motion = bool(cand[4]) if len(cand) > 4 else False
        try:
            members = build_members(tile)
        except ValueError:
            continue   # a grid is not a whole number of such tiles
        try:
            b = Batch(members, tile=tile, j_replicas=reps, j_float=j_float, sort_every=every, ppl=ppl,
                      motion_sort=motion)
        except _lib.PicError:
            continue
        b.capture()
        timings[cand] = time_batch(b, steps)
        if b.check() != 0:
            raise RuntimeError(f"device error while tuning {cand}")
        b.close()
    best = min(timings, key=timings.get)
    return best, timings

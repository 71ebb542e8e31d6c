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
given tile size.

Timing every candidate on the whole batch would take long, so the candidates
are first timed on a sample of the members; but a sample leaves much of the
device idle, where small tiles (more workgroups) look better than they are
once every compute unit is busy.  The few fastest are therefore timed again on
the whole batch (refine), and the fastest of those wins."""
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


def _time_candidate(build_members, cand, steps, j_float):
    """Seconds per step of the batch built for candidate cand, or None when
    the library refuses it or a grid is not a whole number of its tiles."""
    from .sim import Batch
    from . import _lib
    tile, reps, every, ppl = cand[:4]
    motion = bool(cand[4]) if len(cand) > 4 else False
    try:
        members = build_members(tile)
    except ValueError:
        return None
    try:
        b = Batch(members, tile=tile, j_replicas=reps, j_float=j_float, sort_every=every, ppl=ppl,
                  motion_sort=motion)
    except _lib.PicError:
        return None
    del members
    b.capture()
    t = time_batch(b, steps)
    if b.check() != 0:
        raise RuntimeError(f"device error while tuning {cand}")
    b.close()
    return t


def autotune_batch(build_members: Callable[[int], Sequence[dict]],
                   candidates: Sequence[Candidate] = DEFAULT_CANDIDATES,
                   steps: int = 4, j_float: bool = False,
                   refine_members: Callable[[int], Sequence[dict]] = None,
                   refine_top: int = 3) -> Tuple[Candidate, Dict[Candidate, float], Dict[Candidate, float]]:
    """Returns (best candidate, {candidate: seconds per step on
    build_members}, {candidate: seconds per step on refine_members} for the
    refine_top fastest, empty without refine_members); candidates the library
    refuses (LDS budget, a cadence the tile cannot take, particles per lane
    outside the default current) or whose grids are not whole tiles are
    skipped."""
    timings: Dict[Candidate, float] = {}
    for cand in candidates:
        t = _time_candidate(build_members, cand, steps, j_float)
        if t is not None:
            timings[cand] = t
    if not timings:
        raise RuntimeError("no candidate configuration runs this batch")
    refined: Dict[Candidate, float] = {}
    if refine_members is not None:
        for cand in sorted(timings, key=timings.get)[:max(1, refine_top)]:
            t = _time_candidate(refine_members, cand, steps, j_float)
            if t is not None:
                refined[cand] = t
    pool = refined or timings
    best = min(pool, key=pool.get)
    return best, timings, refined

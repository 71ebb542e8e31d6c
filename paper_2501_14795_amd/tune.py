"""Autotuner for the batched mode: times candidate launch configurations
(tile size x LDS current replicas x sort cadence) on graph replays of the
actual batch and keeps the fastest.  The particle arrays must be grouped by
tile for each candidate tile size, so the caller supplies a function that
builds the members' initial states for a given tile size.

The push processes one particle per lane per pass with the next 64-particle
chunk already loading, so particles per lane is not a tuning dimension
here: the sort cadence and the tile size set how much work a workgroup
streams between sorts."""
from __future__ import annotations

import time
from typing import Callable, Dict, Sequence, Tuple

Candidate = Tuple[int, int, int]   # (tile, replicas, sort_every)

DEFAULT_CANDIDATES: Tuple[Candidate, ...] = (
    (8, 1, 1), (8, 1, 2), (16, 1, 1), (16, 2, 1), (16, 1, 2), (16, 1, 4), (32, 1, 1), (32, 1, 2))


def time_batch(batch, steps: int) -> float:
    """Seconds per step of `batch` (graph-replayed if captured), over whole
    sort-cadence cycles after one cycle of warm-up."""
    k = max(1, int(getattr(batch, "sort_every", 1)))
    steps = -(-steps // k) * k
    batch.step(k)
    batch.stream.synchronize()
    t0 = time.perf_counter()
    batch.step(steps)
    batch.stream.synchronize()
    return (time.perf_counter() - t0) / steps


def autotune_batch(build_members: Callable[[int], Sequence[dict]],
                   candidates: Sequence[Candidate] = DEFAULT_CANDIDATES,
                   steps: int = 4, j_float: bool = False) -> Tuple[Candidate, Dict[Candidate, float]]:
    """Returns ((tile, replicas, sort_every), {candidate: seconds per step})."""
    from .sim import Batch
    from . import _lib
    timings: Dict[Candidate, float] = {}
    for tile, reps, every in candidates:
        try:
            members = build_members(tile)
        except ValueError:
            continue   # a grid is not a whole number of such tiles
        try:
            b = Batch(members, tile=tile, j_replicas=reps, j_float=j_float, sort_every=every)
        except _lib.PicError:
            continue   # e.g. over the LDS budget, or a cadence the tile cannot take
        b.capture()
        timings[(tile, reps, every)] = time_batch(b, steps)
        if b.check() != 0:
            raise RuntimeError(f"device error while tuning tile={tile} replicas={reps} sort_every={every}")
        b.close()
    best = min(timings, key=timings.get)
    return best, timings

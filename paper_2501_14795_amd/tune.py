"""Autotuner for the batched mode: times candidate launch configurations
(tile size x LDS current replicas) on graph replays of the actual batch and
keeps the fastest.  The particle arrays must be grouped by tile for each
candidate tile size, so the caller supplies a function that builds the
members' initial states for a given tile size."""
from __future__ import annotations

import time
from typing import Callable, Dict, List, Sequence, Tuple

DEFAULT_CANDIDATES: Tuple[Tuple[int, int], ...] = ((8, 1), (16, 1), (16, 2), (32, 1))


def time_batch(batch, steps: int) -> float:
    """Seconds per step of `batch` (graph-replayed if captured)."""
    import torch
    batch.step(1)
    batch.stream.synchronize()
    t0 = time.perf_counter()
    batch.step(steps)
    batch.stream.synchronize()
    return (time.perf_counter() - t0) / steps


def autotune_batch(build_members: Callable[[int], Sequence[dict]],
                   candidates: Sequence[Tuple[int, int]] = DEFAULT_CANDIDATES,
                   steps: int = 3, j_float: bool = False) -> Tuple[Tuple[int, int], Dict[Tuple[int, int], float]]:
    """Returns ((tile, replicas), {candidate: seconds per step})."""
    from .sim import Batch
    from . import _lib
    timings: Dict[Tuple[int, int], float] = {}
    for tile, reps in candidates:
        try:
            members = build_members(tile)
        except ValueError:
            continue   # a grid is not a whole number of such tiles
        try:
            b = Batch(members, tile=tile, j_replicas=reps, j_float=j_float)
        except _lib.PicError:
            continue   # e.g. over the LDS budget
        b.capture()
        timings[(tile, reps)] = time_batch(b, steps)
        if b.check() != 0:
            raise RuntimeError(f"device error while tuning tile={tile} replicas={reps}")
        b.close()
    best = min(timings, key=timings.get)
    return best, timings

"""Pins of the oracle's strict tile sort (Sec. 4.3, Fig. 4.5).

The canonical result is characterised by four properties, each taken from the
paper's description of the sort: (a) the new sections hold only their own
tile's particles, counted from the final positions (step 1); (b) a particle
already inside its tile's new section is not moved; (c) the holes of a section
are filled by the particles entering that tile (steps 2-5), and -- the
tie-break the paper leaves to atomics, fixed here -- in ascending order of
their old slots; (d) the result is a permutation.  Brute-force enumeration over
all permutations of tiny arrays shows these determine a unique answer, which
the oracle must return.
"""
import itertools
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    d = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split(":")
            vals = [int(t) for t in v.split()]
            d[k.strip()] = vals if len(vals) > 1 or k.strip() in ("ix", "iy", "off", "src", "removed",
                                                                  "off_old") else vals[0]
    return d


@pytest.mark.parametrize("name", ["sort_fig45.txt", "sort_shift3.txt", "sort_window.txt"])
def test_sort_golden(ora, name):
    g = _read_golden(name)
    removed = None if "removed" not in g else np.array(g["removed"], bool)
    off, src = ora.sort_canonical(g["nx"], g["ny"], g["T"], g["ix"], g["iy"], removed=removed)
    assert off.tolist() == g["off"]
    assert src.tolist() == g["src"]


def _tiles(nx, T, ix, iy):
    return (np.asarray(iy) // T) * (nx // T) + np.asarray(ix) // T


def _valid(perm, tile, off):
    n = len(tile)
    for j in range(n):
        t = tile[perm[j]]
        if not (off[t] <= j < off[t + 1]):
            return False
    stay = [off[tile[i]] <= i < off[tile[i] + 1] for i in range(n)]
    for i in range(n):
        if stay[i] and perm[i] != i:
            return False
    for t in range(len(off) - 1):
        filled = [perm[j] for j in range(off[t], off[t + 1]) if not stay[j]]
        if filled != sorted(filled):
            return False
    return True


def test_sort_brute_force_tiny(ora):
    rng = np.random.default_rng(0)
    for trial in range(150):
        nx, ny, T = [(2, 2, 1), (4, 2, 2), (3, 1, 1), (2, 1, 1)][trial % 4]
        n = int(rng.integers(0, 7))
        ix = rng.integers(0, nx, n)
        iy = rng.integers(0, ny, n)
        tile = _tiles(nx, T, ix, iy)
        ntiles = (nx // T) * (ny // T)
        off = np.r_[0, np.cumsum(np.bincount(tile, minlength=ntiles))] if n else np.zeros(ntiles + 1, int)
        sols = [p for p in itertools.permutations(range(n)) if _valid(p, tile, off)]
        assert len(sols) == 1
        o_off, o_src = ora.sort_canonical(nx, ny, T, ix, iy)
        assert o_off.tolist() == off.tolist()
        assert tuple(o_src.tolist()) == sols[0]


def test_sort_properties_large(ora):
    rng = np.random.default_rng(1)
    nx, ny, T = 64, 32, 8
    for n in [0, 1, 1000, 20000]:
        ix = rng.integers(0, nx, n)
        iy = rng.integers(0, ny, n)
        off, src = ora.sort_canonical(nx, ny, T, ix, iy)
        tile = _tiles(nx, T, ix, iy)
        assert sorted(src.tolist()) == list(range(n))
        assert off.tolist() == np.r_[0, np.cumsum(np.bincount(tile, minlength=(nx // T) * (ny // T)))].tolist()
        assert _valid(src, tile, off)


def test_sort_rejects_bad_cells(ora):
    with pytest.raises(ValueError):
        ora.sort_canonical(4, 4, 2, [0, 4], [0, 0])


def _valid_removal(perm, tile, removed, off):
    """(a) sections hold their own tile, (b) a kept particle already inside
    its new section stays, (c) holes take movers in ascending old slot,
    (d) every kept particle appears exactly once and no removed one does."""
    n_new = off[-1]
    kept = [i for i in range(len(tile)) if not removed[i]]
    if sorted(perm) != kept:
        return False
    for j in range(n_new):
        t = tile[perm[j]]
        if not (off[t] <= j < off[t + 1]):
            return False
    stay = [not removed[i] and off[tile[i]] <= i < off[tile[i] + 1] for i in range(len(tile))]
    for i in range(n_new):
        if stay[i] and perm[i] != i:
            return False
    for t in range(len(off) - 1):
        filled = [perm[j] for j in range(off[t], off[t + 1]) if not stay[j]]
        if filled != sorted(filled):
            return False
    return True


def test_sort_with_removal_brute_force_tiny(ora):
    """The moving window's sort: some particles removed, new ones appended;
    enumerating every arrangement of the kept particles shows the properties
    fix one answer, which the oracle returns."""
    rng = np.random.default_rng(7)
    for trial in range(150):
        nx, ny, T = [(2, 2, 1), (4, 2, 2), (3, 1, 1), (2, 1, 1)][trial % 4]
        n = int(rng.integers(1, 7))
        ix = rng.integers(0, nx, n)
        iy = rng.integers(0, ny, n)
        removed = rng.random(n) < 0.3
        tile = _tiles(nx, T, ix, iy)
        ntiles = (nx // T) * (ny // T)
        kept_tiles = tile[~removed]
        off = np.r_[0, np.cumsum(np.bincount(kept_tiles, minlength=ntiles))]
        n_new = int(off[-1])
        sols = [p for p in itertools.permutations(range(n), n_new) if _valid_removal(list(p), tile, removed, off)]
        assert len(sols) == 1, (trial, len(sols))
        o_off, o_src = ora.sort_canonical(nx, ny, T, ix, iy, removed=removed)
        assert o_off.tolist() == off.tolist()
        assert tuple(o_src.tolist()) == sols[0]


def test_stable_grouping_by_tile(ora):
    """sort_stable_by_tile is pinned by the properties that define it
    uniquely: a permutation, tiles non-decreasing along the result, and
    inside each tile the original indices increasing; offsets equal to the
    tile histogram's prefix sums.  Brute force over every permutation of a
    tiny input agrees."""
    rng = np.random.default_rng(3)
    for nx, ny, T, n in ((32, 16, 8, 500), (64, 64, 16, 3000), (16, 16, 16, 40)):
        ix = rng.integers(0, nx, n).astype(np.int32)
        iy = rng.integers(0, ny, n).astype(np.int32)
        off, src = ora.sort_stable_by_tile(nx, ny, T, ix, iy)
        assert sorted(src.tolist()) == list(range(n))
        tile = (iy[src] // T) * (nx // T) + ix[src] // T
        assert (np.diff(tile) >= 0).all()
        same = np.diff(tile) == 0
        assert (np.diff(src)[same] > 0).all()
        counts = np.bincount((iy // T) * (nx // T) + ix // T, minlength=(nx // T) * (ny // T))
        assert np.array_equal(off, np.r_[0, np.cumsum(counts)])
    # brute force: the unique permutation with the defining properties
    ix = np.array([9, 1, 12, 3, 9, 0], np.int32)
    iy = np.array([2, 7, 0, 1, 6, 5], np.int32)
    tile = (iy // 8) * 2 + ix // 8
    ok = [p for p in itertools.permutations(range(6))
          if all(tile[p[k]] < tile[p[k + 1]] or (tile[p[k]] == tile[p[k + 1]] and p[k] < p[k + 1])
                 for k in range(5))]
    assert len(ok) == 1
    assert ora.sort_stable_by_tile(16, 8, 8, ix, iy)[1].tolist() == list(ok[0])
    with pytest.raises(ValueError):
        ora.sort_stable_by_tile(16, 8, 8, np.array([16], np.int32), np.array([0], np.int32))


# ---------------------------------------------------------------- motion-class sort
# The alternative sort of Sec. 4.3 (after Germaschewski et al.): the particles
# are regrouped by their new tile in one counting pass keyed on their motion
# class.  Its result is characterised by: (a) the new sections hold only their
# tile's particles, counted from the final positions; (b) inside a section the
# particles come in ascending motion class, the class of a particle being the
# step (dtx, dty) from its old section's tile to its new tile on the periodic
# tile grid, numbered (dty + 1) * 3 + (dtx + 1), with the step counted +1 on
# an axis of two tiles (both neighbours coincide); (c) within one class, in
# ascending old slot; (d) a permutation.  Brute force over all permutations of
# tiny arrays finds exactly one such order, which the oracle must return.

@pytest.mark.parametrize("name", ["sort_motion_1d.txt", "sort_motion_2d.txt", "sort_motion_two_tiles.txt"])
def test_sort_motion_golden(ora, name):
    g = _read_golden(name)
    off, src = ora.sort_motion_classes(g["nx"], g["ny"], g["T"], g["ix"], g["iy"], g["off_old"])
    assert off.tolist() == g["off"]
    assert src.tolist() == g["src"]


def _step(a, b, m):
    d = (b - a) % m
    return 0 if d == 0 else (1 if d == 1 else (-1 if d == m - 1 else None))


def _motion_valid(perm, new_tile, cls, off):
    for j, i in enumerate(perm):
        if not (off[new_tile[i]] <= j < off[new_tile[i] + 1]):
            return False
    for t in range(len(off) - 1):
        sec = [perm[j] for j in range(off[t], off[t + 1])]
        keys = [(cls[i], i) for i in sec]
        if keys != sorted(keys):
            return False
    return True


def test_sort_motion_brute_force_tiny(ora):
    rng = np.random.default_rng(1)
    for trial in range(120):
        nx, ny, T = [(3, 3, 1), (4, 2, 2), (2, 2, 1), (6, 2, 2), (3, 1, 1)][trial % 5]
        ntx, nty = nx // T, ny // T
        ntiles = ntx * nty
        n = int(rng.integers(0, 7))
        # old sections: a random split of the n slots over the tiles
        sizes = np.bincount(rng.integers(0, ntiles, n), minlength=ntiles) if n else np.zeros(ntiles, int)
        off_old = np.r_[0, np.cumsum(sizes)]
        old_tile = np.repeat(np.arange(ntiles), sizes)
        # every particle ends in its section's tile or a neighbour (cells anywhere inside it)
        ix = np.zeros(n, int)
        iy = np.zeros(n, int)
        new_tile = np.zeros(n, int)
        cls = np.zeros(n, int)
        for i in range(n):
            sx, sy = old_tile[i] % ntx, old_tile[i] // ntx
            tx = (sx + int(rng.integers(-1, 2))) % ntx
            ty = (sy + int(rng.integers(-1, 2))) % nty
            ix[i] = tx * T + int(rng.integers(0, T))
            iy[i] = ty * T + int(rng.integers(0, T))
            new_tile[i] = ty * ntx + tx
            cls[i] = (_step(sy, ty, nty) + 1) * 3 + (_step(sx, tx, ntx) + 1)
        off = np.r_[0, np.cumsum(np.bincount(new_tile, minlength=ntiles))] if n else np.zeros(ntiles + 1, int)
        sols = [p for p in itertools.permutations(range(n)) if _motion_valid(p, new_tile, cls, off)]
        assert len(sols) == 1
        o_off, o_src = ora.sort_motion_classes(nx, ny, T, ix, iy, off_old)
        assert o_off.tolist() == off.tolist()
        assert tuple(o_src.tolist()) == sols[0]


def test_sort_motion_rejects_moves_beyond_a_neighbour(ora):
    # 4 tiles along x: from tile 0 to tile 2 is two tiles
    with pytest.raises(ValueError):
        ora.sort_motion_classes(8, 2, 2, [4], [0], [0, 1, 1, 1, 1])
    with pytest.raises(ValueError):
        ora.sort_motion_classes(8, 2, 2, [8], [0], [0, 1, 1, 1, 1])   # outside the grid

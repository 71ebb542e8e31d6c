"""Sort cadence (pic_config.sort_every = k > 1) on the GPU against the oracle.

The particles are re-sorted every k-th step; in between, a particle may be up
to k - 1 cells outside the tile whose section holds it, and the push stages a
halo k cells wide.  The particle values do not depend on when the sort runs,
and the canonical sort depends only on the slot order it starts from, so the
oracle replays every step from the GPU's own state: positions within 1e-5
cells, momenta within 1e-5 of max|u|, J within 1e-5 of max|J|, and at every
k-th step the sort bit-exact against the oracle's canonical sort of the GPU's
cells.  Fast particles (up to 0.7 cells per step) on small grids with two
tiles per axis make particles leave their tiles by several cells and across
the periodic seam.  Free runs: fields within 1e-5 of the oracle's after 12
steps, continuity within 1e-6 at every push, Gauss's law kept; batched
members bit-identical to standalone runs with the same cadence, also when a
step count is not a whole number of cycles.  Guards: a push beyond the
cadence without a sort, and a sort with nothing to sort."""
import numpy as np
import pytest

import pic_workloads as pw
from _parity import (flush, make_pair, matched_particle_errors, oracle_from_gpu, particle_errors, rel_err,
                     sort_replay, species_states)

pytestmark = pytest.mark.gpu

DX = DY = 0.1
DT = 0.07


def _lib():
    from paper_2501_14795_amd import _lib
    return _lib


def _fast(nspecies=1):
    """Relativistic drifting species: up to 0.7 cells per step in x and y."""
    drifts = [(2.0, -1.5, 0.5), (-1.8, 1.2, -0.3)]
    return [pw.SpeciesSpec(-1.0, (2, 2), (0.6, 0.6, 0.3), drifts[k]) for k in range(nspecies)]


def _outside(sim, species, tile):
    """Largest distance, in cells, of a particle outside the tile whose
    section holds it (periodic)."""
    g = sim.state(species)
    off = sim.tile_offsets(species)
    ntx = sim.nx // tile
    sec = np.repeat(np.arange(len(off) - 1), np.diff(off))
    gx0, gy0 = (sec % ntx) * tile, (sec // ntx) * tile

    def dist(i, g0, n):
        d = (i - g0) % n                      # 0 .. n-1 to the right of the tile start
        right = np.where(d >= tile, d - tile + 1, 0)
        left = np.where(d >= tile, n - d, 0)
        return np.minimum(right, left)
    return int(max(dist(g["ix"], gx0, sim.nx).max(initial=0), dist(g["iy"], gy0, sim.ny).max(initial=0)))


@pytest.mark.parametrize("nx,ny,tile,k,nspecies,esirkepov", [
    (32, 32, 16, 4, 1, False),    # two tiles per axis: the periodic seam is a tile border
    (64, 32, 16, 2, 2, False),
    (64, 64, 8, 2, 1, False),
    (96, 64, 32, 2, 1, False),
    (32, 48, 16, 4, 1, True),
    (64, 64, 32, 4, 1, False),    # 32 x 32 tiles with a 4-cell pad (one workgroup per CU)
])
def test_cadence_replay(nx, ny, tile, k, nspecies, esirkepov):
    specs = _fast(nspecies)
    states = species_states(nx, ny, tile, specs, 5)
    E, B = pw.random_fields(nx, ny, 0.05, 5)
    sim, _ = make_pair(nx, ny, DX, DY, DT, tile, specs, states, E, B, esirkepov=esirkepov, sort_every=k)
    worst = [0.0, 0.0, 0.0]
    out_max = 0
    for step in range(3 * k):
        out_max = max(out_max, _outside(sim, 0, tile))
        ref = oracle_from_gpu(sim, specs, DX, DY, DT)
        ref.esirkepov = esirkepov
        ref.push_deposit()
        sim.push_deposit()
        assert sim.check() == 0
        for s in range(nspecies):
            pos, du = particle_errors(sim.state(s), ref.species[s], nx, ny)
            worst[0], worst[1] = max(worst[0], pos), max(worst[1], du)
        worst[2] = max(worst[2], rel_err(sim.field_arrays()["J"], ref.J))
        if step % k == k - 1:
            sort_replay(sim, specs, tile)
            assert _outside(sim, 0, tile) == 0
        sim.field_advance()
    flush(f"T{tile} k={k} x{nspecies} esirkepov={esirkepov}: pos {worst[0]:.2e} u {worst[1]:.2e} "
          f"J {worst[2]:.2e}; particles up to {out_max} cells outside their tile at a push")
    assert worst[0] < 1e-5 and worst[1] < 1e-5 and worst[2] < 1e-5
    assert out_max >= min(k - 1, 2)
    sim.close()


@pytest.mark.parametrize("k", [2, 4])
def test_cadence_free_run(k):
    L = _lib()
    nx = ny = 64
    specs = _fast()
    states = species_states(nx, ny, 16, specs, 8)
    sim, ora = make_pair(nx, ny, DX, DY, DT, 16, specs, states, sort_every=k)
    g0 = None
    worst = 0.0
    for step in range(12):
        sim.diag(L.PIC_DIAG_RHO_SNAPSHOT)
        sim.push_deposit()
        d = sim.diag(L.PIC_DIAG_CONTINUITY)
        worst = max(worst, d.continuity_max / d.rho_max)
        if step % k == k - 1:
            sim.sort()
        sim.field_advance()
        ora.step(T=16)
        if step == 0:
            g0 = sim.diag(L.PIC_DIAG_GAUSS).gauss_max
    assert sim.check() == 0
    f = sim.field_arrays()
    errs = {c: rel_err(f[c], getattr(ora, c)) for c in ("E", "B", "J")}
    pos, du, _ = matched_particle_errors(sim.state(0), ora.species[0], nx, ny)
    g = sim.diag(L.PIC_DIAG_GAUSS).gauss_max
    flush(f"k={k} 12 steps: {errs} pos {pos:.2e} u {du:.2e}; continuity {worst:.2e}; gauss {g0:.2e} -> {g:.2e}")
    assert max(errs.values()) <= 1e-5
    assert pos < 1e-5 and du < 1e-5
    assert worst <= 1e-6
    assert g < 2e-5
    sim.close()


def test_cadence_step_equals_explicit_calls():
    """pic_step with sort_every = 4 is the explicit sequence with a sort after
    every fourth push, bit for bit."""
    nx = ny = 64
    specs = _fast()
    states = species_states(nx, ny, 16, specs, 9)
    a, _ = make_pair(nx, ny, DX, DY, DT, 16, specs, states, sort_every=4)
    b, _ = make_pair(nx, ny, DX, DY, DT, 16, specs, states, sort_every=4)
    for step in range(10):
        a.step()
        b.push_deposit()
        if step % 4 == 3:
            b.sort()
        b.field_advance()
    assert a.check() == 0 and b.check() == 0
    assert np.array_equal(a.tile_offsets(0), b.tile_offsets(0))
    sa, sb = a.state(0), b.state(0)
    for name in sa:
        assert np.array_equal(sa[name], sb[name]), name
    fa, fb = a.field_arrays(), b.field_arrays()
    for name in fa:
        assert np.array_equal(fa[name], fb[name]), name
    a.close()
    b.close()


@pytest.mark.parametrize("k,steps", [(2, 5), (4, 7)])
def test_cadence_batch_equals_standalone(k, steps):
    from paper_2501_14795_amd import Batch, Sim
    members = pw.batched_members(n_sims=6, seed=17)
    specs = []
    for m in members:
        st = pw.species_state(m["nx"], m["ny"], 16, m["spec"], m["seed"])
        specs.append(dict(nx=m["nx"], ny=m["ny"], dx=m["dx"], dy=m["dy"], dt=m["dt"],
                          species=[(m["spec"].qm, m["spec"].q, st)]))
    captured = Batch(specs, tile=16, sort_every=k)
    captured.capture()
    direct = Batch(specs, tile=16, sort_every=k)
    # a partial cycle first, then whole cycles from the graph, then a partial one
    for n in (1, steps, 2):
        captured.step(n)
        direct.step(n)
    total = 1 + steps + 2
    assert captured.check() == 0 and direct.check() == 0
    for i, m in enumerate(specs):
        s = Sim(m["nx"], m["ny"], m["dx"], m["dy"], m["dt"], 16, m["species"], sort_every=k)
        for _ in range(total):
            s.step()
        fs = s.field_arrays()
        ps = s.state(0)
        for b in (captured, direct):
            fb = b[i].field_arrays()
            for c in ("E", "B", "J"):
                assert np.array_equal(fb[c], fs[c]), (i, c)
            pb = b[i].state(0)
            for a in ("cell", "x", "y", "ux", "uy", "uz"):
                assert np.array_equal(pb[a], ps[a]), (i, a)
        s.close()
    flush(f"k={k}: {len(specs)} members, {total} steps, captured and direct batches equal standalone runs")
    captured.close()
    direct.close()


def test_cadence_guards():
    from paper_2501_14795_amd import PicError
    L = _lib()
    nx = ny = 32
    specs = _fast()
    states = species_states(nx, ny, 16, specs, 3)
    sim, _ = make_pair(nx, ny, DX, DY, DT, 16, specs, states, sort_every=2)
    sim.sort()                       # nothing to sort: no-op
    assert sim.check() == 0
    sim.push_deposit()
    sim.push_deposit()
    with pytest.raises(PicError) as e:   # a third push could leave the staged halo
        sim.push_deposit()
    assert e.value.code == L.PIC_EORDER
    sim.sort()
    sim.sort()                       # the second finds nothing to do
    sim.push_deposit()
    assert sim.check() == 0
    sim.close()
    one, _ = make_pair(nx, ny, DX, DY, DT, 16, specs, states)
    one.push_deposit()
    with pytest.raises(PicError) as e:
        one.push_deposit()
    assert e.value.code == L.PIC_EORDER
    one.close()

"""The alternative sort (PIC_FLAG_FULL_SORT; the full re-sort of Sec. 4.3):
after every push the particles are regrouped out of place by a stable sort
on the tile id.  Bit-exact against the oracle's stable grouping of the GPU's
post-push state (every array and tile_offset), with one and two species, at
T = 8, 16, 32 and with a sort cadence of 2; free runs within the usual
tolerances of the oracle; the same physics as the in-place sort (fields
within round-off after 10 steps, particles paired by nearest neighbour)."""
import numpy as np
import pytest

import oracle
import pic_workloads as pw
from _parity import (flush, make_pair, matched_particle_errors, oracle_from_gpu, particle_errors, rel_err,
                     species_states)

pytestmark = pytest.mark.gpu

DX = DY = 0.1
DT = 0.07
ARRAYS = ("ix", "iy", "x", "y", "ux", "uy", "uz")


def _specs(nspecies):
    drifts = [(0.6, -0.4, 0.2), (-0.5, 0.3, 0.0)]
    return [pw.SpeciesSpec(-1.0, (3, 3), (0.3, 0.3, 0.3), drifts[k]) for k in range(nspecies)]


@pytest.mark.parametrize("nx,ny,tile,nspecies,every", [(64, 64, 16, 1, 1), (96, 64, 32, 2, 1), (64, 32, 8, 1, 2)])
def test_full_sort_replay(nx, ny, tile, nspecies, every):
    specs = _specs(nspecies)
    states = species_states(nx, ny, tile, specs, 6)
    E, B = pw.random_fields(nx, ny, 0.05, 6)
    sim, _ = make_pair(nx, ny, DX, DY, DT, tile, specs, states, E, B, sort_every=every, full_sort=True)
    worst = [0.0, 0.0, 0.0]
    for step in range(3 * every):
        ref = oracle_from_gpu(sim, specs, DX, DY, DT)
        ref.push_deposit()
        sim.push_deposit()
        assert sim.check() == 0
        for k in range(nspecies):
            pos, du = particle_errors(sim.state(k), ref.species[k], nx, ny)
            worst[0], worst[1] = max(worst[0], pos), max(worst[1], du)
        worst[2] = max(worst[2], rel_err(sim.field_arrays()["J"], ref.J))
        if step % every == every - 1:
            pre = [sim.state(k) for k in range(nspecies)]
            sim.sort()
            assert sim.check() == 0
            for k in range(nspecies):
                off, src = oracle.sort_stable_by_tile(nx, ny, tile, pre[k]["ix"], pre[k]["iy"])
                post = sim.state(k)
                for a in ARRAYS:
                    assert np.array_equal(post[a], pre[k][a][src]), a
                assert np.array_equal(sim.tile_offsets(k), off)
        sim.field_advance()
    flush(f"full sort T{tile} x{nspecies} k={every}: pos {worst[0]:.2e} u {worst[1]:.2e} J {worst[2]:.2e}; "
          f"regrouping bit-exact")
    assert worst[0] < 1e-5 and worst[1] < 1e-5 and worst[2] < 1e-5
    sim.close()


def test_full_sort_free_run_matches_oracle_and_in_place_sort():
    nx = ny = 64
    specs = _specs(1)
    states = species_states(nx, ny, 16, specs, 7)
    full, ora = make_pair(nx, ny, DX, DY, DT, 16, specs, states, full_sort=True)
    inplace, _ = make_pair(nx, ny, DX, DY, DT, 16, specs, states)
    for _ in range(10):
        full.step()
        inplace.step()
        ora.step(T=16)
    assert full.check() == 0 and inplace.check() == 0
    ff, fi = full.field_arrays(), inplace.field_arrays()
    e_ora = {c: rel_err(ff[c], getattr(ora, c)) for c in ("E", "B", "J")}
    e_in = {c: rel_err(ff[c], fi[c].astype(np.float64)) for c in ("E", "B", "J")}
    pos, du, _ = matched_particle_errors(full.state(0), ora.species[0], nx, ny)
    flush(f"full sort, 10 steps: vs oracle {e_ora}, vs in-place sort {e_in}; particles {pos:.2e} {du:.2e}")
    assert max(e_ora.values()) <= 1e-5 and max(e_in.values()) <= 1e-5
    assert pos < 1e-5 and du < 1e-5
    full.close()
    inplace.close()

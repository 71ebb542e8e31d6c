"""Four species of both signs and different charge-to-mass ratios and
densities -- electrons, positrons, heavy ions (q/m = 1/100, a tenth of the
density) and a fast electron beam -- on the GPU against the oracle: every
species' push replayed from the GPU's state (positions within 1e-5 cells,
momenta within 1e-5 of max|u|), the summed current within 1e-5 of max|J|,
each species' sort bit-exact; 10 free-running steps with every field within
1e-5 of the oracle's; the continuity residual of the total charge at
round-off (1e-6 of the gross charge density sum_s |q_s| n_s).  The fixed-point current scales every species by the largest
|q|, so species whose charges differ in sign and size share one accumulator."""
import numpy as np
import pytest

import pic_workloads as pw
from _parity import (flush, make_pair, matched_particle_errors, oracle_from_gpu, particle_errors, rel_err,
                     sort_replay, species_states)

pytestmark = pytest.mark.gpu

DX = DY = 0.1
DT = 0.07

SPECS = [
    pw.SpeciesSpec(-1.0, (2, 2), (0.1, 0.1, 0.1), (0.0, 0.0, 0.0)),
    pw.SpeciesSpec(1.0, (2, 2), (0.1, 0.1, 0.1), (0.0, 0.0, 0.2)),
    pw.SpeciesSpec(0.01, (1, 2), (0.01, 0.01, 0.01), (0.0, 0.0, 0.0), n0=0.1),
    pw.SpeciesSpec(-1.0, (1, 1), (0.05, 0.05, 0.05), (1.5, 0.5, 0.0), n0=0.3),
]
GROSS = sum(s.n0 for s in SPECS)   # sum_s |q_s| n_s per cell


@pytest.mark.parametrize("tile", [16, 32])
def test_four_species_replay(tile):
    nx, ny = 64, 64
    states = species_states(nx, ny, tile, SPECS, 21)
    E, B = pw.random_fields(nx, ny, 0.05, 21)
    sim, _ = make_pair(nx, ny, DX, DY, DT, tile, SPECS, states, E, B)
    worst = [0.0, 0.0, 0.0]
    for _ in range(3):
        ref = oracle_from_gpu(sim, SPECS, DX, DY, DT)
        ref.push_deposit()
        sim.push_deposit()
        assert sim.check() == 0
        for k in range(len(SPECS)):
            pos, du = particle_errors(sim.state(k), ref.species[k], nx, ny)
            worst[0], worst[1] = max(worst[0], pos), max(worst[1], du)
        worst[2] = max(worst[2], rel_err(sim.field_arrays()["J"], ref.J))
        sort_replay(sim, SPECS, tile)
        sim.field_advance()
    flush(f"four species T{tile}: pos {worst[0]:.2e} u {worst[1]:.2e} J {worst[2]:.2e}")
    assert worst[0] < 1e-5 and worst[1] < 1e-5 and worst[2] < 1e-5
    sim.close()


def test_four_species_free_run_and_continuity():
    from paper_2501_14795_amd import _lib as L
    nx = ny = 64
    states = species_states(nx, ny, 16, SPECS, 22)
    sim, ora = make_pair(nx, ny, DX, DY, DT, 16, SPECS, states)
    worst = worst_abs = 0.0
    for _ in range(10):
        sim.diag(L.PIC_DIAG_RHO_SNAPSHOT)
        sim.push_deposit()
        d = sim.diag(L.PIC_DIAG_CONTINUITY)
        worst = max(worst, d.continuity_max / d.rho_max)
        worst_abs = max(worst_abs, d.continuity_max)
        sim.sort()
        sim.field_advance()
        ora.step(T=16)
    assert sim.check() == 0
    f = sim.field_arrays()
    errs = {c: rel_err(f[c], getattr(ora, c)) for c in ("E", "B", "J")}
    pe = [matched_particle_errors(sim.state(k), ora.species[k], nx, ny)[:2] for k in range(len(SPECS))]
    d = sim.diag(L.PIC_DIAG_ENERGY)
    ue, ub, uk = ora.energies()
    ek = max(abs(d.u_k[k] - uk[k]) / abs(uk[k]) for k in range(len(SPECS)))
    flush(f"four species, 10 steps: {errs}; particles {pe}; continuity {worst_abs:.2e} = {worst:.2e} of the net "
          f"max|rho|, {worst_abs / GROSS:.2e} of the gross density; kinetic energy {ek:.2e}")
    assert max(errs.values()) <= 1e-5
    assert all(p < 1e-5 and u < 1e-5 for p, u in pe)
    # the residual comes from rounding each species' current, so it scales
    # with the gross charge density sum_s |q_s| n_s (2.4 per cell here), not
    # with the net density the diagnostic's rho_max measures (about 0.2)
    assert worst_abs <= 1e-6 * GROSS
    assert ek <= 1e-5
    sim.close()

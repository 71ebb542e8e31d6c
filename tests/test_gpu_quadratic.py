"""The quadratic particle shape (PIC_FLAG_QUADRATIC: the gather at each
component's staggered point and Esirkepov's current with the second-order
B-spline) on the GPU against the FP64 oracle's quadratic shape, with the
tolerances of the default deposit's parity tests: one step from the GPU's own
state -- positions within 1e-5 cells, momenta within 1e-5 of max|u|, J within
1e-5 of max|J|, the sort bit-exact -- at T = 8, 16, 32 (the halo pad is 2);
10 free-running steps -- fields within 1e-5; the device continuity residual
with the quadratic charge within 1e-6 of max|rho| and Gauss's law kept;
batched members bit-identical to standalone runs; at the 2048^2 workload,
continuity at round-off and the total current equal to the charge moved; grids
of one tile on an axis; and with the motion-class sort, fields bit-identical to
the in-place sort's."""
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


def _specs(nspecies=1, u_th=0.1, drift=(0.0, 0.0, 0.0), ppc=(4, 4)):
    return [pw.SpeciesSpec(-1.0, ppc, (u_th,) * 3, drift if k == 0 else tuple(-v for v in drift))
            for k in range(nspecies)]


@pytest.mark.parametrize("tile,nspecies", [(16, 1), (8, 2), (32, 1)])
def test_quadratic_replay(tile, nspecies):
    nx = ny = 64
    specs = _specs(nspecies, u_th=0.2, drift=(0.3, -0.2, 0.1))
    states = species_states(nx, ny, tile, specs, 71)
    E, B = pw.random_fields(nx, ny, 0.05, 71)
    sim, _ = make_pair(nx, ny, DX, DY, DT, tile, specs, states, E, B, quadratic=True)
    worst = [0.0, 0.0, 0.0]
    for step in range(3):
        ref = oracle_from_gpu(sim, specs, DX, DY, DT)
        ref.quadratic = True
        ref.push_deposit()
        sim.push_deposit()
        assert sim.check() == 0
        for k in range(nspecies):
            pos, du = particle_errors(sim.state(k), ref.species[k], nx, ny)
            worst[0], worst[1] = max(worst[0], pos), max(worst[1], du)
        worst[2] = max(worst[2], rel_err(sim.field_arrays()["J"], ref.J))
        sort_replay(sim, specs, tile)
        sim.field_advance()
    flush(f"quadratic T{tile} x{nspecies}: pos {worst[0]:.2e} u {worst[1]:.2e} J {worst[2]:.2e}")
    assert worst[0] < 1e-5 and worst[1] < 1e-5 and worst[2] < 1e-5
    sim.close()


def test_quadratic_ten_steps():
    w = pw.WORKLOADS["uniform64"]
    states = pw.workload_state(w)
    E, B = pw.random_fields(w.nx, w.ny, 0.05, 72)
    sim, ora = make_pair(w.nx, w.ny, w.dx, w.dy, w.dt, w.tile, w.species, states, E, B, quadratic=True)
    for _ in range(10):
        sim.step()
        ora.step(T=w.tile)
    assert sim.check() == 0
    f = sim.field_arrays()
    errs = {k: rel_err(f[k], getattr(ora, k)) for k in ("E", "B", "J")}
    pos, du, _ = matched_particle_errors(sim.state(0), ora.species[0], w.nx, w.ny)
    flush(f"quadratic 10 steps: {errs} pos {pos:.2e} u {du:.2e}")
    assert max(errs.values()) <= 1e-5
    assert pos < 1e-5 and du < 1e-5
    sim.close()


def test_quadratic_continuity_gauss_and_difference_from_linear():
    L = _lib()
    nx = ny = 64
    specs = _specs(u_th=0.2, drift=(0.2, 0.1, 0.0))
    states = species_states(nx, ny, 16, specs, 73)
    sim, _ = make_pair(nx, ny, DX, DY, DT, 16, specs, states, quadratic=True)
    lin, _ = make_pair(nx, ny, DX, DY, DT, 16, specs, states, esirkepov=True)
    sim.push_deposit()
    lin.push_deposit()
    d = rel_err(sim.field_arrays()["J"], lin.field_arrays()["J"].astype(np.float64))
    flush(f"quadratic vs linear Esirkepov current after one step: {d:.2e}")
    assert d > 1e-3
    sim.sort()
    sim.field_advance()
    g0 = sim.diag(L.PIC_DIAG_GAUSS).gauss_max
    worst = 0.0
    for _ in range(20):
        sim.diag(L.PIC_DIAG_RHO_SNAPSHOT)
        sim.push_deposit()
        dd = sim.diag(L.PIC_DIAG_CONTINUITY)
        worst = max(worst, dd.continuity_max / dd.rho_max)
        sim.sort()
        sim.field_advance()
    g = sim.diag(L.PIC_DIAG_GAUSS).gauss_max
    flush(f"quadratic continuity worst {worst:.2e}; gauss {g0:.2e} -> {g:.2e}")
    assert worst <= 1e-6
    assert g < 2e-5
    assert sim.check() == 0
    sim.close()
    lin.close()


def test_quadratic_batch_equals_standalone():
    from paper_2501_14795_amd import Batch, Sim
    members = pw.batched_members(n_sims=5, seed=74)
    specs = []
    for m in members:
        st = pw.species_state(m["nx"], m["ny"], 16, m["spec"], m["seed"])
        specs.append(dict(nx=m["nx"], ny=m["ny"], dx=m["dx"], dy=m["dy"], dt=m["dt"],
                          species=[(m["spec"].qm, m["spec"].q, st)]))
    b = Batch(specs, tile=16, quadratic=True)
    b.capture()
    b.step(4)
    assert b.check() == 0
    for i, m in enumerate(specs):
        s = Sim(m["nx"], m["ny"], m["dx"], m["dy"], m["dt"], 16, m["species"], quadratic=True)
        for _ in range(4):
            s.step()
        fb, fs = b[i].field_arrays(), s.field_arrays()
        for k in ("E", "B", "J"):
            assert np.array_equal(fb[k], fs[k]), (i, k)
        pb, ps = b[i].state(0), s.state(0)
        for a in ("cell", "x", "y", "ux", "uy", "uz"):
            assert np.array_equal(pb[a], ps[a]), (i, a)
        s.close()
    b.close()


def test_quadratic_full_size_continuity():
    """The 2048^2 bench workload (67 M particles) with the quadratic shape:
    continuity at round-off with the quadratic charge, and the total current
    equal to the charge moved."""
    from paper_2501_14795_amd import Sim
    L = _lib()
    w = pw.WORKLOADS["warm2048"]
    st = pw.workload_state(w)[0]
    spec = w.species[0]
    sim = Sim(w.nx, w.ny, w.dx, w.dy, w.dt, w.tile, [(spec.qm, spec.q, st)], quadratic=True)
    del st
    for _ in range(2):
        sim.step()
    pre = sim.state(0)
    sim.diag(L.PIC_DIAG_RHO_SNAPSHOT)
    sim.push_deposit()
    d = sim.diag(L.PIC_DIAG_CONTINUITY)
    post = sim.state(0)
    J = sim.field_arrays()["J"]
    dX = (post["ix"] - pre["ix"]).astype(np.float64) + (post["x"].astype(np.float64) - pre["x"])
    dX = (dX + w.nx / 2) % w.nx - w.nx / 2
    want = spec.q * dX.sum()
    got = J[0].astype(np.float64).sum() * w.dt / w.dx
    flush(f"quadratic 2048^2: continuity {d.continuity_max / d.rho_max:.2e}; sum Jx dt/dx {got:.6e} vs {want:.6e}")
    assert d.continuity_max <= 1e-6 * d.rho_max
    assert abs(got - want) <= 1e-8 * abs(spec.q) * pre["ix"].size
    assert sim.check() == 0
    sim.close()


@pytest.mark.parametrize("nx,ny,tile", [(16, 16, 16), (16, 32, 16), (48, 8, 8)])
def test_quadratic_degenerate_tile_grids(nx, ny, tile):
    """One tile on an axis (the tile's own halo folds onto its periodic
    images at both ends, two nodes deep) and a one-tile-high strip: replay
    against the oracle within 1e-5, the sort bit-exact."""
    specs = _specs(1, u_th=0.25, drift=(0.3, -0.3, 0.1))
    states = species_states(nx, ny, tile, specs, 75)
    E, B = pw.random_fields(nx, ny, 0.05, 75)
    sim, _ = make_pair(nx, ny, DX, DY, DT, tile, specs, states, E, B, quadratic=True)
    worst = [0.0, 0.0, 0.0]
    for step in range(3):
        ref = oracle_from_gpu(sim, specs, DX, DY, DT)
        ref.quadratic = True
        ref.push_deposit()
        sim.push_deposit()
        assert sim.check() == 0
        pos, du = particle_errors(sim.state(0), ref.species[0], nx, ny)
        worst[0], worst[1] = max(worst[0], pos), max(worst[1], du)
        worst[2] = max(worst[2], rel_err(sim.field_arrays()["J"], ref.J))
        sort_replay(sim, specs, tile)
        sim.field_advance()
    flush(f"quadratic {nx}x{ny} T{tile}: pos {worst[0]:.2e} u {worst[1]:.2e} J {worst[2]:.2e}")
    assert worst[0] < 1e-5 and worst[1] < 1e-5 and worst[2] < 1e-5
    sim.close()


def test_quadratic_with_the_motion_class_sort():
    """The quadratic shape with the motion-class sort (its copy back then
    runs as its own pass): fields bit-identical to the in-place sort's after
    six steps (the fixed-point current does not depend on particle order),
    and within 1e-5 of the oracle."""
    from paper_2501_14795_amd import Sim
    nx = ny = 64
    specs = _specs(1, u_th=0.2, drift=(0.2, 0.1, 0.0))
    states = species_states(nx, ny, 16, specs, 76)
    E, B = pw.random_fields(nx, ny, 0.05, 76)
    motion, ora = make_pair(nx, ny, DX, DY, DT, 16, specs, states, E, B, quadratic=True, motion_sort=True)
    inplace = Sim(nx, ny, DX, DY, DT, 16, [(s.qm, s.q, st) for s, st in zip(specs, states)], E=E, B=B,
                  quadratic=True)
    for _ in range(6):
        motion.step()
        inplace.step()
        ora.step(T=16)
    assert motion.check() == 0 and inplace.check() == 0
    fm, fi = motion.field_arrays(), inplace.field_arrays()
    for k in ("E", "B", "J"):
        assert np.array_equal(fm[k], fi[k]), k
    errs = {k: rel_err(fm[k], getattr(ora, k)) for k in ("E", "B", "J")}
    flush(f"quadratic + motion-class sort, 6 steps: bit-identical to the in-place sort; vs oracle {errs}")
    assert max(errs.values()) <= 1e-5
    motion.close()
    inplace.close()

"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (the workload's tile, default current mode), and with a sort cadence of 2.

Every step is replayed by the oracle over ALL particles from the GPU's own
pre-step state and E/B fields (about 8 s of FP64 per 67M-particle step):
  * push + move: every particle, slot by slot -- position within 1e-5 cells
    (X = ix + x modulo the box), momentum within 1e-5 of max|u|, and every
    offset in [0, 1);
  * current: every J node, per component within 1e-5 of that component's
    max|J|; also the discrete continuity residual (device FP64 diagnostic)
    and the total current, sum(Jx) dt/dx = sum_p q dX_p;
  * sort: the oracle's canonical sort of ALL the GPU's post-push cells,
    compared bit for bit with the GPU's sorted arrays and tile_offset.
"""
import time

import numpy as np
import pytest

import oracle
import pic_workloads as pw
from _parity import PARTICLE_ARRAYS, flush, particle_errors

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _lib():
    from paper_2501_14795_amd import _lib
    return _lib


def _full_push_errors(pre_list, post_list, specs, E, B, w):
    """The oracle's push + deposit of every particle from the GPU's pre-step
    state; returns (worst position error, worst relative momentum error,
    per-component J errors relative to each component's max|J|, oracle J)."""
    osp = [oracle.OracleSpecies(s.qm, s.q, pre["ix"], pre["iy"], pre["x"], pre["y"], pre["ux"], pre["uy"],
                                pre["uz"]) for s, pre in zip(specs, pre_list)]
    ora = oracle.OracleSim(w.nx, w.ny, w.dx, w.dy, w.dt, osp, E, B)
    ora.push_deposit()
    pos = du = 0.0
    for o, post in zip(osp, post_list):
        p, u = particle_errors(post, o, w.nx, w.ny)
        pos, du = max(pos, p), max(du, u)
    return pos, du, ora.J


def _total_current_check(pre_list, post_list, specs, J, w):
    """sum(Jx) dt/dx = sum_p q dX_p, likewise y; dX from the GPU's own positions."""
    for comp, (a, c) in enumerate((("ix", "x"), ("iy", "y"))):
        n = w.nx if comp == 0 else w.ny
        cell_size = w.dx if comp == 0 else w.dy
        want = 0.0
        for pre, post, s in zip(pre_list, post_list, specs):
            d = (post[a] - pre[a]).astype(np.float64) + (post[c].astype(np.float64) - pre[c])
            d = (d + n / 2) % n - n / 2
            want += s.q * d.sum()
        got = J[comp].astype(np.float64).sum() * w.dt / cell_size
        scale = sum(abs(s.q) for s in specs) * sum(p[a].size for p in pre_list) * 1e-2
        assert abs(got - want) <= 1e-6 * scale, (comp, got, want)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name,steps,every", [("warm2048", 2, 1), ("weibel512", 2, 1), ("warm2048", 4, 2)])
def test_full_size_step(name, steps, every):
    """every > 1: the sort cadence -- the sort (checked bit-exact over all
    particles) after every second push only."""
    from paper_2501_14795_amd import Sim
    L = _lib()
    w = pw.WORKLOADS[name]
    t0 = time.time()
    states = pw.workload_state(w)
    sim = Sim(w.nx, w.ny, w.dx, w.dy, w.dt, w.tile, [(s.qm, s.q, st) for s, st in zip(w.species, states)],
              sort_every=every)
    del states
    flush(f"[{name}] initialised {sim.n_tiles} tiles in {time.time() - t0:.1f}s")
    for step in range(steps):
        pre = [sim.state(k) for k in range(len(w.species))]
        f = sim.field_arrays()
        E, B = f["E"].astype(np.float64), f["B"].astype(np.float64)
        del f
        sim.diag(L.PIC_DIAG_RHO_SNAPSHOT)
        sim.push_deposit()
        d = sim.diag(L.PIC_DIAG_CONTINUITY | L.PIC_DIAG_COUNTS)
        assert d.continuity_max <= 1e-6 * d.rho_max, (d.continuity_max, d.rho_max)
        post = [sim.state(k) for k in range(len(w.species))]
        for g in post:
            assert (g["x"] >= 0).all() and (g["x"] < 1).all() and (g["y"] >= 0).all() and (g["y"] < 1).all()
        J = sim.field_arrays()["J"]
        _total_current_check(pre, post, w.species, J, w)
        t1 = time.time()
        pos, du, Jo = _full_push_errors(pre, post, w.species, E, B, w)
        ej = [float(np.abs(J[c] - Jo[c]).max() / max(np.abs(Jo[c]).max(), 1e-30)) for c in range(3)]
        n = sum(p["ix"].size for p in pre)
        flush(f"[{name}] step {step}: oracle over all {n} particles in {time.time() - t1:.1f}s: "
              f"pos {pos:.2e} u {du:.2e} J {ej[0]:.2e} {ej[1]:.2e} {ej[2]:.2e}; "
              f"continuity {d.continuity_max:.2e}; leavers {list(d.leavers)[:len(w.species)]}")
        assert pos < TOL and du < TOL and max(ej) < TOL
        del pre, Jo, E, B
        if step % every != every - 1:
            del post
            sim.field_advance()
            continue
        # the sort, bit-exact over all particles
        sim.sort()
        assert sim.check() == 0
        for k in range(len(w.species)):
            srt = sim.state(k)
            off, src = oracle.sort_canonical(w.nx, w.ny, w.tile, post[k]["ix"], post[k]["iy"])
            assert np.array_equal(sim.tile_offsets(k), off)
            for a in PARTICLE_ARRAYS:
                assert np.array_equal(srt[a], post[k][a][src]), a
            moved = int((src != np.arange(src.size)).sum())
            flush(f"[{name}] step {step} species {k}: sort bit-exact, {moved} particles moved")
            del srt, off, src
        del post
        sim.field_advance()
    assert sim.check() == 0
    sim.close()
    flush(f"[{name}] done in {time.time() - t0:.1f}s")

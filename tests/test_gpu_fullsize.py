"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (the workload's tile, default current mode), and with a sort cadence of 2.

The oracle cannot run every particle of a 67M-particle step in a test, so:
  * push + move: a seeded random sample of particles is advanced one by one by
    the oracle from the GPU's own pre-step state and full E/B fields and
    compared element by element (same tolerances as the small cases);
  * sort: the oracle's canonical sort of ALL the GPU's post-push cells is
    compared bit for bit with the GPU's sorted arrays and tile_offset;
  * current: properties that hold at any size -- the discrete continuity
    residual (device FP64 diagnostic) and the total current, sum(Jx) dt/dx =
    sum_p q dX_p over all particles (dX from the GPU's own positions).
"""
import time

import numpy as np
import pytest

import oracle
import pic_workloads as pw
from _parity import PARTICLE_ARRAYS, flush

pytestmark = pytest.mark.gpu

SAMPLE = 20000


def _lib():
    from paper_2501_14795_amd import _lib
    return _lib


def _sampled_push_errors(pre, post, idx, spec, E, B, w):
    st = {k: pre[k][idx] for k in ("ix", "iy", "x", "y", "ux", "uy", "uz")}
    osp = oracle.OracleSpecies(spec.qm, spec.q, st["ix"], st["iy"], st["x"], st["y"], st["ux"], st["uy"], st["uz"])
    ora = oracle.OracleSim(w.nx, w.ny, w.dx, w.dy, w.dt, [osp], E, B)
    ora.push_deposit()
    X = post["ix"][idx] + post["x"][idx].astype(np.float64)
    Y = post["iy"][idx] + post["y"][idx].astype(np.float64)
    dX = (X - (osp.ix + osp.x) + w.nx / 2) % w.nx - w.nx / 2
    dY = (Y - (osp.iy + osp.y) + w.ny / 2) % w.ny - w.ny / 2
    umax = max(np.abs(osp.ux).max(), np.abs(osp.uy).max(), np.abs(osp.uz).max())
    du = max(np.abs(post["ux"][idx] - osp.ux).max(), np.abs(post["uy"][idx] - osp.uy).max(),
             np.abs(post["uz"][idx] - osp.uz).max())
    return max(np.abs(dX).max(), np.abs(dY).max()), du / umax


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
    rng = np.random.default_rng(123)
    for step in range(steps):
        pre = [sim.state(k) for k in range(len(w.species))]
        f = sim.field_arrays()
        E, B = f["E"].astype(np.float64), f["B"].astype(np.float64)
        sim.diag(L.PIC_DIAG_RHO_SNAPSHOT)
        sim.push_deposit()
        d = sim.diag(L.PIC_DIAG_CONTINUITY | L.PIC_DIAG_COUNTS)
        assert d.continuity_max <= 1e-6 * d.rho_max, (d.continuity_max, d.rho_max)
        post = [sim.state(k) for k in range(len(w.species))]
        J = sim.field_arrays()["J"]
        _total_current_check(pre, post, w.species, J, w)
        for k, spec in enumerate(w.species):
            idx = rng.choice(pre[k]["ix"].size, SAMPLE, replace=False)
            pos, du = _sampled_push_errors(pre[k], post[k], idx, spec, E, B, w)
            flush(f"[{name}] step {step} species {k}: sampled pos {pos:.2e} u {du:.2e}; "
                  f"continuity {d.continuity_max:.2e}; leavers {d.leavers[k]}")
            assert pos < 1e-5 and du < 1e-5
        del pre
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

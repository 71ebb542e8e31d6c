"""The moving window (the last step of Listing 3.1) on the GPU against the
oracle.

The oracle's window step is the definition: E, B and every particle move one
cell towards -x, window column 0's particles leave, new particles come in at
column nx - 1, then the canonical sort.  The GPU keeps the shift as a
relabelling of the periodic array columns (window column i = array column
(i + origin) mod nx), so after each GPU move:

* in window columns, E and B equal the oracle's bit for bit, and the
  particles equal the oracle's as a multiset, bit for bit (their order follows
  the array's tiles, not the window's);
* in array columns, every particle array and tile_offset equal the oracle's
  canonical sort of the GPU's state before the move, with the particles of
  the origin column removed and the new ones (moved into that column)
  appended -- the exact layout, bit for bit.

Steps between the moves are the ordinary periodic steps; one replayed step
after several moves matches the oracle's step in window columns to the usual
tolerances, and the continuity residual of a push right after a move stays at
round-off.  Checkpoint / resume carries the counts and the origin.  Error
paths: too many new particles for the capacity, a new particle outside the
last window column, a simulation without the moving-window flag, a bad origin
in a loaded state."""
import numpy as np
import pytest

import oracle
import pic_workloads as pw
from _parity import flush, particle_errors, rel_err

pytestmark = pytest.mark.gpu

DX = DY = 0.1
DT = 0.07
ARRAYS = ("ix", "iy", "x", "y", "ux", "uy", "uz")


def _lib():
    from paper_2501_14795_amd import _lib
    return _lib


def _setup(nx, ny, tile, nspecies=1, seed=3, **options):
    from paper_2501_14795_amd import Sim
    specs = [pw.SpeciesSpec(-1.0, (2, 2), (0.15,) * 3, (0.1, 0.05 * k, 0.0)) for k in range(nspecies)]
    states = [pw.species_state(nx, ny, tile, s, seed, k) for k, s in enumerate(specs)]
    E, B = pw.random_fields(nx, ny, 0.05, seed)
    cap = [st["ix"].size + 8 * ny * 4 for st in states]
    sim = Sim(nx, ny, DX, DY, DT, tile, [(s.qm, s.q, st) for s, st in zip(specs, states)], E=E, B=B,
              moving_window=True, capacity=cap, **options)
    return sim, specs, states, E, B, cap


def _column(nx, ny, tile, spec, seed, k):
    """New plasma for window column nx - 1, grouped by tile."""
    return pw.species_state(nx, ny, tile, spec, seed, k, cell_box=(nx - 1, nx, 0, ny))


def _window_oracle(sim, specs, j_filter=0, esirkepov=False):
    """OracleSim holding the GPU's state in window columns (GPU slot order)."""
    f = sim.window_fields()
    osp = []
    for k, s in enumerate(specs):
        g = sim.window_state(k)
        osp.append(oracle.OracleSpecies(s.qm, s.q, g["ix"], g["iy"], g["x"], g["y"], g["ux"], g["uy"], g["uz"]))
    return oracle.OracleSim(sim.nx, sim.ny, DX, DY, DT, osp, f["E"].astype(np.float64), f["B"].astype(np.float64),
                            j_filter=j_filter, esirkepov=esirkepov)


def _sorted_rows(d):
    """The particles as rows (ix, iy, x, y, ux, uy, uz) in lexicographic order."""
    cols = [np.asarray(d[a], np.float64) for a in ARRAYS]
    order = np.lexsort(cols[::-1])
    return np.stack([c[order] for c in cols])


def _expected_layout(pre, inject, origin, nx, ny, tile):
    """The oracle's canonical sort, in array columns, of the state before the
    move with the origin column's particles removed and the new particles
    (moved into the origin column) appended."""
    cat = {a: np.r_[pre[a], inject[a]] for a in ARRAYS}
    cat["ix"] = np.r_[pre["ix"], np.full(inject["ix"].size, origin, np.int32)].astype(np.int32)
    removed = np.r_[pre["ix"] == origin, np.zeros(inject["ix"].size, bool)]
    off, src = oracle.sort_canonical(nx, ny, tile, cat["ix"], cat["iy"], removed=removed)
    return {a: v[src] for a, v in cat.items()}, np.asarray(off, np.int64)


@pytest.mark.parametrize("nx,ny,tile,nspecies,options", [
    (64, 32, 16, 1, {}), (48, 40, 8, 2, {}), (96, 64, 32, 1, {}),
    # with the current filter, the Esirkepov deposit and the full re-sort between moves
    (64, 48, 16, 2, {"j_filter": 1, "esirkepov": True, "motion_sort": True}),
])
def test_window_step_matches_oracle(nx, ny, tile, nspecies, options):
    L = _lib()
    sim, specs, *_ = _setup(nx, ny, tile, nspecies, **options)
    oopt = {"j_filter": options.get("j_filter", 0), "esirkepov": options.get("esirkepov", False)}
    n0 = sim.counts()
    cycles = 5
    for cycle in range(cycles):
        for _ in range(2):
            sim.step()
        assert sim.check() == 0
        origin = sim.window_origin()
        assert origin == cycle % nx
        pre = [sim.state(k) for k in range(nspecies)]
        ref = _window_oracle(sim, specs)
        inject = [_column(nx, ny, tile, s, 100 + cycle, k) for k, s in enumerate(specs)]
        ref.move_window(inject, tile)
        # odd cycles hand over device-resident copies instead of host arrays
        sim.move_window([sim.upload_particles(c) for c in inject] if cycle & 1 else inject)
        assert sim.window_origin() == (origin + 1) % nx
        f = sim.window_fields()
        assert np.array_equal(f["E"].astype(np.float64), ref.E)
        assert np.array_equal(f["B"].astype(np.float64), ref.B)
        counts = sim.counts()
        for k in range(nspecies):
            o = ref.species[k]
            assert counts[k] == o.ix.size
            want = {a: getattr(o, a) for a in ARRAYS}
            assert np.array_equal(_sorted_rows(sim.window_state(k)), _sorted_rows(want))
            lay, off = _expected_layout(pre[k], inject[k], origin, nx, ny, tile)
            g = sim.state(k)
            for a in ARRAYS:
                assert np.array_equal(g[a], lay[a]), a
            assert np.array_equal(sim.tile_offsets(k), off)
        flush(f"T{tile} cycle {cycle}: origin {origin} -> {sim.window_origin()}, counts {counts} (start {n0}), "
              f"window step bit-exact")
    # one step after the moves against the oracle's step in window columns
    ref = _window_oracle(sim, specs, **oopt)
    ref.push_deposit()
    sim.push_deposit()
    assert sim.check() == 0
    pos = du = 0.0
    for k in range(nspecies):
        p, u = particle_errors(sim.window_state(k), ref.species[k], nx, ny)
        pos, du = max(pos, p), max(du, u)
    ej = rel_err(sim.window_fields()["J"], ref.J)
    flush(f"T{tile}: step after {cycles} moves: pos {pos:.2e} u {du:.2e} J {ej:.2e}")
    assert pos < 1e-5 and du < 1e-5 and ej < 1e-5
    sim.sort()
    sim.field_advance()
    # a push right after a window move conserves charge as usual
    sim.move_window([_column(nx, ny, tile, s, 999, k) for k, s in enumerate(specs)])
    sim.diag(L.PIC_DIAG_RHO_SNAPSHOT)
    sim.push_deposit()
    d = sim.diag(L.PIC_DIAG_CONTINUITY)
    assert d.continuity_max <= 1e-6 * d.rho_max
    sim.sort()
    sim.field_advance()
    assert sim.check() == 0
    sim.close()


def test_window_checkpoint_resume():
    """A checkpoint taken after window moves (counts and origin changed)
    resumes in a fresh simulation bit for bit."""
    from paper_2501_14795_amd import Sim
    nx, ny, tile = 64, 32, 16
    sim, specs, states, E, B, cap = _setup(nx, ny, tile)
    for c in range(3):
        sim.step()
        sim.move_window([_column(nx, ny, tile, specs[0], 50 + c, 0)])
    ck = sim.get_state()
    assert ck["window_origin"] == 3 and ck["species"][0]["cell"].size == sim.counts()[0]
    fresh = Sim(nx, ny, DX, DY, DT, tile, [(specs[0].qm, specs[0].q, states[0])], E=E, B=B,
                moving_window=True, capacity=cap)
    fresh.set_state(ck)
    assert fresh.window_origin() == 3 and fresh.counts() == sim.counts()
    for s in (sim, fresh):
        for c in range(2):
            s.step()
            s.move_window([_column(nx, ny, tile, specs[0], 80 + c, 0)])
            s.step()
    a, b = sim.get_state(), fresh.get_state()
    assert a["window_origin"] == b["window_origin"] == 5
    assert np.array_equal(a["fields"], b["fields"])
    for name in ("cell", "x", "y", "ux", "uy", "uz"):
        assert np.array_equal(a["species"][0][name], b["species"][0][name]), name
    sim.close()
    fresh.close()


def test_window_errors():
    from paper_2501_14795_amd import PicError, Sim
    L = _lib()
    nx, ny, tile = 32, 16, 16
    sim, specs, *_ = _setup(nx, ny, tile)
    cap_room = 8 * ny * 4
    col = _column(nx, ny, tile, specs[0], 7, 0)
    big = {k: np.concatenate([v] * (cap_room // v.size + 2)) for k, v in col.items()}
    with pytest.raises(PicError) as e:
        sim.move_window([big])
    assert e.value.code == L.PIC_EINVAL
    wrong = {k: v.copy() for k, v in col.items()}
    wrong["ix"][:] = nx - 2
    before = sim.get_state()
    with pytest.raises(PicError) as e:
        sim.move_window([wrong])
    assert e.value.code == L.PIC_EORDER
    after = sim.get_state()      # a rejected move changes nothing
    assert after["window_origin"] == before["window_origin"] == 0
    assert np.array_equal(after["fields"], before["fields"])
    assert np.array_equal(after["species"][0]["cell"], before["species"][0]["cell"])
    sim.move_window([col])      # a valid move still works afterwards
    sim.step()
    assert sim.check() == 0
    bad = sim.get_state()
    bad["window_origin"] = nx
    with pytest.raises(PicError) as e:
        sim.set_state(bad)
    assert e.value.code == L.PIC_EINVAL
    sim.close()
    st = pw.species_state(nx, ny, tile, specs[0], 1)
    plain = Sim(nx, ny, DX, DY, DT, tile, [(specs[0].qm, specs[0].q, st)])
    with pytest.raises(PicError) as e:
        plain.move_window([col])
    assert e.value.code == L.PIC_EINVAL
    s0 = plain.get_state()
    s0["window_origin"] = 1     # no origin without the moving window
    with pytest.raises(PicError) as e:
        plain.set_state(s0)
    assert e.value.code == L.PIC_EINVAL
    plain.close()


def test_window_full_size():
    """The 2048^2 benchmark workload (67 M particles, 32 x 32 tiles) with the
    moving window: after two steps, one move with a fresh column of plasma.
    In array columns every particle array and tile_offset equal the oracle's
    canonical sort with the origin column removed and the new particles
    appended; E and B change in the origin column only (to zero)."""
    from paper_2501_14795_amd import Sim
    w = pw.WORKLOADS["warm2048"]
    T = w.tile
    spec = w.species[0]
    st = pw.workload_state(w)[0]
    n0 = st["ix"].size
    sim = Sim(w.nx, w.ny, w.dx, w.dy, w.dt, T, [(spec.qm, spec.q, st)], moving_window=True,
              capacity=[n0 + 4 * w.ny * 16])
    del st
    for _ in range(2):
        sim.step()
    pre = sim.state(0)
    f0 = sim.field_arrays()
    col = pw.species_state(T, w.ny, T, spec, 77, 0, cell_box=(T - 1, T, 0, w.ny))
    col["ix"] = col["ix"] + (w.nx - T)
    sim.move_window([col])
    assert sim.check() == 0 and sim.window_origin() == 1
    lay, off = _expected_layout(pre, col, 0, w.nx, w.ny, T)
    del pre
    g = sim.state(0)
    assert sim.counts()[0] == lay["ix"].size
    for a in ARRAYS:
        assert np.array_equal(g[a], lay[a]), a
    assert np.array_equal(sim.tile_offsets(0), off)
    f = sim.field_arrays()
    for c in ("E", "B"):
        assert not f[c][:, :, 0].any()
        assert np.array_equal(f[c][:, :, 1:], f0[c][:, :, 1:]), c
    flush(f"2048^2 window move: {n0} -> {lay['ix'].size} particles, layout bit-exact")
    sim.step()
    assert sim.check() == 0
    sim.close()

"""The moving window (the last step of Listing 3.1) on the GPU against the
oracle.  A window step moves data and re-sorts it canonically, so the GPU must
agree with the oracle's window step applied to the GPU's own state bit for
bit: E and B, every particle array (the particles that left are gone, the new
ones placed) and tile_offset.  Steps between the window moves are the
ordinary GPU steps (their parity is covered elsewhere); the continuity
residual of a push right after a window move stays at round-off.  Error
paths: too many new particles for the capacity, a new particle outside the
last column, a simulation without the moving-window flag."""
import numpy as np
import pytest

import pic_workloads as pw
from _parity import PARTICLE_ARRAYS, flush, oracle_from_gpu

pytestmark = pytest.mark.gpu

DX = DY = 0.1
DT = 0.07


def _lib():
    from paper_2501_14795_amd import _lib
    return _lib


def _setup(nx, ny, tile, nspecies=1, seed=3):
    from paper_2501_14795_amd import Sim
    specs = [pw.SpeciesSpec(-1.0, (2, 2), (0.15,) * 3, (0.1, 0.05 * k, 0.0)) for k in range(nspecies)]
    states = [pw.species_state(nx, ny, tile, s, seed, k) for k, s in enumerate(specs)]
    E, B = pw.random_fields(nx, ny, 0.05, seed)
    cap = [st["ix"].size + 8 * ny * 4 for st in states]
    sim = Sim(nx, ny, DX, DY, DT, tile, [(s.qm, s.q, st) for s, st in zip(specs, states)], E=E, B=B,
              moving_window=True, capacity=cap)
    return sim, specs


def _column(nx, ny, tile, spec, seed, k):
    return pw.species_state(nx, ny, tile, spec, seed, k, cell_box=(nx - 1, nx, 0, ny))


@pytest.mark.parametrize("nx,ny,tile,nspecies", [(64, 32, 16, 1), (48, 40, 8, 2), (96, 64, 32, 1)])
def test_window_step_matches_oracle(nx, ny, tile, nspecies):
    L = _lib()
    sim, specs = _setup(nx, ny, tile, nspecies)
    n0 = sim.counts()
    for cycle in range(4):
        for _ in range(2):
            sim.step()
        assert sim.check() == 0
        ref = oracle_from_gpu(sim, specs, DX, DY, DT)
        inject = [_column(nx, ny, tile, s, 100 + cycle, k) for k, s in enumerate(specs)]
        ref.move_window(inject, tile)
        sim.move_window(inject)
        f = sim.field_arrays()
        assert np.array_equal(f["E"].astype(np.float64), ref.E)
        assert np.array_equal(f["B"].astype(np.float64), ref.B)
        counts = sim.counts()
        for k in range(nspecies):
            g = sim.state(k)
            o = ref.species[k]
            assert counts[k] == o.ix.size
            assert np.array_equal(g["ix"], o.ix) and np.array_equal(g["iy"], o.iy)
            for a in ("x", "y", "ux", "uy", "uz"):
                assert np.array_equal(g[a].astype(np.float64), getattr(o, a)), a
            tiles = (o.iy // tile) * (nx // tile) + o.ix // tile
            want_off = np.r_[0, np.cumsum(np.bincount(tiles, minlength=sim.n_tiles))]
            assert np.array_equal(sim.tile_offsets(k), want_off)
        flush(f"T{tile} cycle {cycle}: counts {counts} (start {n0}), window step bit-exact")
    # a push right after a window move conserves charge as usual
    sim.diag(L.PIC_DIAG_RHO_SNAPSHOT)
    sim.push_deposit()
    d = sim.diag(L.PIC_DIAG_CONTINUITY)
    assert d.continuity_max <= 1e-6 * d.rho_max
    sim.sort()
    sim.field_advance()
    assert sim.check() == 0
    sim.close()


def test_window_errors():
    from paper_2501_14795_amd import PicError, Sim
    L = _lib()
    nx, ny, tile = 32, 16, 16
    sim, specs = _setup(nx, ny, tile)
    cap_room = 8 * ny * 4
    col = _column(nx, ny, tile, specs[0], 7, 0)
    big = {k: np.concatenate([v] * (cap_room // v.size + 2)) for k, v in col.items()}
    with pytest.raises(PicError) as e:
        sim.move_window([big])
    assert e.value.code == L.PIC_EINVAL
    wrong = {k: v.copy() for k, v in col.items()}
    wrong["ix"][:] = nx - 2
    with pytest.raises(PicError) as e:
        sim.move_window([wrong])
    assert e.value.code == L.PIC_EORDER
    sim.move_window([col])      # a valid move still works afterwards
    sim.step()
    assert sim.check() == 0
    sim.close()
    st = pw.species_state(nx, ny, tile, specs[0], 1)
    plain = Sim(nx, ny, DX, DY, DT, tile, [(specs[0].qm, specs[0].q, st)])
    with pytest.raises(PicError) as e:
        plain.move_window([col])
    assert e.value.code == L.PIC_EINVAL
    plain.close()

"""Particles given in any order are grouped by tile on the device (pic_init,
pic_set_state; Sec. 4.1, Fig. 4.3) by a stable radix sort on the tile id:
bit-exact against the oracle's stable grouping (every particle array and
tile_offset), for 1, 2 and 3 radix passes (up to 131,072 tiles), one and
many 16,384-particle chunks, several species, and an already grouped input,
which stays as it is.  The grouped simulation then steps like one started
grouped."""
import numpy as np
import pytest

import oracle
import pic_workloads as pw
from _parity import flush

pytestmark = pytest.mark.gpu

DX = DY = 0.1
DT = 0.07
ARRAYS = ("ix", "iy", "x", "y", "ux", "uy", "uz")


def _shuffled(nx, ny, tile, spec, seed, k=0, how="shuffle"):
    st = pw.species_state(nx, ny, tile, spec, seed, k)
    n = st["ix"].size
    order = np.random.default_rng(seed + 7).permutation(n) if how == "shuffle" else np.arange(n)[::-1]
    return {a: np.ascontiguousarray(v[order]) for a, v in st.items()}


def _check(sim, given, tile, k=0):
    _, src = oracle.sort_stable_by_tile(sim.nx, sim.ny, tile, given["ix"], given["iy"])
    g = sim.state(k)
    for a in ARRAYS:
        assert np.array_equal(g[a], given[a][src]), a
    tiles = (given["iy"] // tile) * (sim.nx // tile) + given["ix"] // tile
    assert np.array_equal(sim.tile_offsets(k),
                          np.r_[0, np.cumsum(np.bincount(tiles, minlength=sim.n_tiles))])


@pytest.mark.parametrize("nx,ny,tile,ppc,how", [
    (32, 32, 16, (1, 1), "reverse"),        # 4 tiles, one chunk, one pass
    (256, 256, 8, (4, 4), "shuffle"),       # 1,024 tiles: two passes, 64 chunks
    (4096, 2048, 8, (1, 1), "shuffle"),     # 131,072 tiles: three passes, 512 chunks
])
def test_init_groups_by_tile(nx, ny, tile, ppc, how):
    from paper_2501_14795_amd import Sim
    spec = pw.SpeciesSpec(-1.0, ppc, (0.1, 0.1, 0.1))
    given = _shuffled(nx, ny, tile, spec, 4, how=how)
    sim = Sim(nx, ny, DX, DY, DT, tile, [(spec.qm, spec.q, given)])
    _check(sim, given, tile)
    sim.step()
    assert sim.check() == 0
    flush(f"{nx} x {ny}, T{tile}, {given['ix'].size} particles ({how}): grouped bit-exact, one step ok")
    sim.close()


def test_init_groups_several_species_and_keeps_grouped_input():
    from paper_2501_14795_amd import Sim
    nx = ny = 64
    specs = [pw.SpeciesSpec(-1.0, (3, 3), (0.1,) * 3), pw.SpeciesSpec(-1.0, (2, 2), (0.1,) * 3)]
    grouped = pw.species_state(nx, ny, 16, specs[0], 2, 0)
    mixed = _shuffled(nx, ny, 16, specs[1], 3, 1)
    sim = Sim(nx, ny, DX, DY, DT, 16, [(specs[0].qm, specs[0].q, grouped), (specs[1].qm, specs[1].q, mixed)])
    g0 = sim.state(0)
    for a in ARRAYS:
        assert np.array_equal(g0[a], grouped[a]), a   # stable: already grouped input is left as it is
    _check(sim, mixed, 16, 1)
    # the grouped simulation steps bit for bit like one started from the grouped particles
    st1 = sim.state(1)
    ref = Sim(nx, ny, DX, DY, DT, 16, [(specs[0].qm, specs[0].q, grouped),
                                        (specs[1].qm, specs[1].q, {a: st1[a] for a in ARRAYS})])
    for _ in range(3):
        sim.step()
        ref.step()
    fa, fb = sim.field_arrays(), ref.field_arrays()
    for c in fa:
        assert np.array_equal(fa[c], fb[c]), c
    sim.close()
    ref.close()

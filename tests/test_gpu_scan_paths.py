"""The sort's recount and scan take two launches up to 64 scan blocks of 256
tiles (each block adds its predecessors' totals itself) and three above
(a separate scan of the block totals).  Both paths, at and just past the
boundary, with many tiles: pic_sort bit-exact against the oracle's canonical
sort of the GPU's own post-push cells, and pic_step (whose sort leaves the
hole fill to the next push) bit-identical to a twin that sorts eagerly."""
import numpy as np
import pytest

import pic_workloads as pw
from _parity import flush, sort_replay

pytestmark = pytest.mark.gpu

DX = DY = 0.1
DT = 0.07


@pytest.mark.parametrize("nx,ny", [(1024, 1024), (1040, 1024), (2048, 1024)])
def test_scan_paths(nx, ny):
    from paper_2501_14795_amd import Sim
    T = 8
    n_tiles = (nx // T) * (ny // T)
    blocks = -(-n_tiles // 256)
    spec = pw.SpeciesSpec(-1.0, (1, 1), (0.3, 0.3, 0.1), (0.2, -0.1, 0.0))
    state = pw.species_state(nx, ny, T, spec, 41)
    sim = Sim(nx, ny, DX, DY, DT, T, [(spec.qm, spec.q, state)])
    twin = Sim(nx, ny, DX, DY, DT, T, [(spec.qm, spec.q, state)])
    # the separate calls, the sort checked against the oracle
    sim.push_deposit()
    sort_replay(sim, [spec], T)
    sim.field_advance()
    twin.push_deposit()
    twin.sort()
    twin.field_advance()
    # then pic_step against the separate calls, two steps
    for _ in range(2):
        sim.step()
        twin.push_deposit()
        twin.sort()
        twin.field_advance()
        a, b = sim.state(0), twin.state(0)
        for k in a:
            assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(sim.tile_offsets(0), twin.tile_offsets(0))
    assert sim.check() == 0 and twin.check() == 0
    flush(f"{nx}x{ny}, T{T}: {n_tiles} tiles, {blocks} scan blocks "
          f"({'two' if blocks <= 64 else 'three'} launches): sort bit-exact, pic_step equal to the separate calls")
    sim.close()
    twin.close()

"""pic_step captured into a HIP graph by the caller (torch's graph capture on
the simulation's stream) and replayed: with the default options, the current
filter, the Esirkepov deposit and the full re-sort, every replay -- with eager
work and synchronisations of the program in between -- leaves exactly the
state (fields, particles, tile_offset) that the same number of eager steps of
a twin simulation leaves.  Nothing in the captured step is a memset node or
a synchronisation."""
import numpy as np
import pytest

import pic_workloads as pw
from _parity import flush, species_states

pytestmark = pytest.mark.gpu

DX = DY = 0.1
DT = 0.07


def _same(a, b):
    fa, fb = a.field_arrays(), b.field_arrays()
    for c in fa:
        assert np.array_equal(fa[c], fb[c]), c
    sa, sb = a.state(0), b.state(0)
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k
    assert np.array_equal(a.tile_offsets(0), b.tile_offsets(0))


@pytest.mark.parametrize("options", [{}, {"j_filter": 2}, {"esirkepov": True}, {"motion_sort": True}])
def test_captured_step_replays_like_eager_steps(options):
    import torch
    from paper_2501_14795_amd import Sim, _lib
    nx = ny = 64
    spec = pw.SpeciesSpec(-1.0, (3, 3), (0.2, 0.2, 0.2), (0.3, -0.2, 0.1))
    state = species_states(nx, ny, 16, [spec], 12)[0]
    E, B = pw.random_fields(nx, ny, 0.05, 12)
    side = torch.cuda.Stream()
    graphed = Sim(nx, ny, DX, DY, DT, 16, [(spec.qm, spec.q, state)], E=E, B=B, stream=side, **options)
    eager = Sim(nx, ny, DX, DY, DT, 16, [(spec.qm, spec.q, state)], E=E, B=B, **options)
    graphed.step()            # one eager step first (as torch's capture examples warm up)
    eager.step()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        _lib.pic_step(graphed.handle, side.cuda_stream)
    # the capture recorded the step without running it
    _same(graphed, eager)
    junk = torch.zeros(1 << 20, device="cuda")
    for rep in range(4):
        g.replay()
        eager.step()
        junk.add_(1.0)            # the program's own eager work between replays
        torch.cuda.synchronize()
        _same(graphed, eager)
        flush(f"{options or 'default'}: replay {rep} equals the eager step")
    assert graphed.check() == 0 and eager.check() == 0
    del g
    graphed.close()
    eager.close()

"""pic_step runs the sort on the caller's stream and the field half (J fold,
filter, field advance) on the library's second stream, joined back before it
returns.  The two halves touch disjoint data, so the result must be exactly
that of the same kernels one after the other: a twin stepped through the
separate entry points (pic_push_deposit, pic_sort, pic_field_advance, all on
one stream) must hold bit-identical fields, particles and tile offsets after
every step -- on the default stream and on a caller stream, with the filter,
with a sort cadence of 2 (whose unsorted steps take the unforked path), and
with the motion-class sort, also for a species of only 144 particles.  The
forked simulation's particles are read through state(), which completes the
hole fill its sort left to the next push (pic_sync)."""
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


@pytest.mark.parametrize("options,caller_stream", [
    ({}, False),
    ({}, True),
    ({"j_filter": 2}, True),
    ({"sort_every": 2}, False),
    ({"motion_sort": True}, True),
    ({"motion_sort": True, "tiny": True}, False),
])
def test_forked_step_equals_the_sequential_calls(options, caller_stream):
    import torch
    from paper_2501_14795_amd import Sim
    options = dict(options)
    tiny = options.pop("tiny", False)
    nx = ny = 64
    spec = pw.SpeciesSpec(-1.0, (3, 3), (0.2, 0.2, 0.2), (0.3, -0.2, 0.1))
    if tiny:   # 16 cells x 9 particles
        state = pw.species_state(nx, ny, 16, spec, 21, cell_box=(0, 4, 0, 4))
        assert state["ix"].size == 144
    else:
        state = species_states(nx, ny, 16, [spec], 21)[0]
    E, B = pw.random_fields(nx, ny, 0.05, 21)
    stream = torch.cuda.Stream() if caller_stream else None
    forked = Sim(nx, ny, DX, DY, DT, 16, [(spec.qm, spec.q, state)], E=E, B=B, stream=stream, **options)
    serial = Sim(nx, ny, DX, DY, DT, 16, [(spec.qm, spec.q, state)], E=E, B=B, **options)
    every = options.get("sort_every", 1)
    for k in range(6):
        forked.step()
        serial.push_deposit()
        if (k + 1) % every == 0:
            serial.sort()
        serial.field_advance()
        torch.cuda.synchronize()
        _same(forked, serial)
    flush(f"{options or 'default'}{' (144 particles)' if tiny else ''}, caller stream {caller_stream}: "
          "six steps equal the sequential calls")
    assert forked.check() == 0 and serial.check() == 0
    forked.close()
    serial.close()

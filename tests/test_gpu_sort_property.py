"""Property test of the GPU sort (hypothesis): random small configurations --
tile 8, 16 or 32, one to four tiles per axis, a random rectangle of loaded
cells (ragged and empty tiles), 1 to 9 particles per cell, momenta up to
relativistic in any direction, sort cadence 1 or 2 -- pushed and then sorted
on the GPU; the sort must equal the oracle's canonical sort of the GPU's own
post-push cells bit for bit (every array and tile_offset)."""
import numpy as np
import pytest

hypothesis = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

import pic_workloads as pw  # noqa: E402
from _parity import sort_replay  # noqa: E402

pytestmark = pytest.mark.gpu


@st.composite
def configs(draw):
    T = draw(st.sampled_from([8, 16, 32]))
    nx = T * draw(st.integers(1, 4))
    ny = T * draw(st.integers(1, 4))
    x0 = draw(st.integers(0, nx - 1))
    x1 = draw(st.integers(x0 + 1, nx))
    y0 = draw(st.integers(0, ny - 1))
    y1 = draw(st.integers(y0 + 1, ny))
    ppc = (draw(st.integers(1, 3)), draw(st.integers(1, 3)))
    u_th = draw(st.sampled_from([0.01, 0.2, 0.8]))
    drift = tuple(draw(st.floats(-1.5, 1.5)) for _ in range(3))
    every = draw(st.sampled_from([1, 2]))
    seed = draw(st.integers(0, 10_000))
    return T, nx, ny, (x0, x1, y0, y1), ppc, u_th, drift, every, seed


@settings(max_examples=30, deadline=None, derandomize=True, database=None)
@given(configs())
def test_gpu_sort_matches_oracle_on_random_configs(cfg):
    from paper_2501_14795_amd import Sim
    T, nx, ny, box, ppc, u_th, drift, every, seed = cfg
    spec = pw.SpeciesSpec(-1.0, ppc, (u_th,) * 3, drift)
    state = pw.species_state(nx, ny, T, spec, seed, cell_box=box)
    E, B = pw.random_fields(nx, ny, 0.05, seed)
    sim = Sim(nx, ny, 0.1, 0.1, 0.07, T, [(spec.qm, spec.q, state)], E=E, B=B, sort_every=every)
    for step in range(every):
        sim.push_deposit()
        assert sim.check() == 0
        if step < every - 1:
            sim.field_advance()
    sort_replay(sim, [spec], T)
    sim.close()

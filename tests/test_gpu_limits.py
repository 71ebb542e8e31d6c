"""Limits of the GPU path, on the GPU against the oracle.

* The fixed-point current with very many contributions to one node: 70,000
  and 250,000 particles in one cell.  The int64 sums stay exact, so J differs
  from the oracle by no more than the rounding of each contribution (the FP32
  product, 2^-24 of it, then a truncation to 2^-30 of the largest possible
  contribution) times the number of contributions, plus the FP32 rounding of
  J.  (Earlier versions of the accumulator overflowed beyond 2^16
  contributions per node and tile; the 64-bit sums now hold any count below
  2^31 particles per tile.)
* The largest grid extents (cell index packed as ix | iy << 16, so
  nx, ny <= 32767): one replayed step on a 32752 x 16 and a 16 x 32752 grid
  with particles crossing the periodic seam -- particles, J and the sort
  against the oracle.
"""
import numpy as np
import pytest

import pic_workloads as pw
from _parity import flush, oracle_from_gpu, particle_errors, rel_err, sort_replay

pytestmark = pytest.mark.gpu

DX = DY = 0.1
DT = 0.07


def _crowd(n, seed):
    rng = np.random.default_rng(seed)
    return {"ix": np.full(n, 5, np.int32), "iy": np.full(n, 6, np.int32),
            "x": rng.uniform(0.3, 0.7, n).astype(np.float32), "y": rng.uniform(0.3, 0.7, n).astype(np.float32),
            "ux": (0.01 * rng.standard_normal(n)).astype(np.float32),
            "uy": (0.01 * rng.standard_normal(n)).astype(np.float32),
            "uz": (0.01 * rng.standard_normal(n)).astype(np.float32)}


@pytest.mark.parametrize("n", [70000, 250000])
def test_fixed_point_many_contributions(n):
    from paper_2501_14795_amd import Sim
    spec = pw.SpeciesSpec(-1.0, (4, 4))
    st = _crowd(n, n)
    sim = Sim(32, 32, DX, DY, DT, 16, [(spec.qm, spec.q, st)])
    ref = oracle_from_gpu(sim, [spec], DX, DY, DT)
    ref.push_deposit()
    sim.push_deposit()
    assert sim.check() == 0
    J = sim.field_arrays()["J"].astype(np.float64)
    for c, unit in enumerate((abs(spec.q) * DX / DT, abs(spec.q) * DY / DT, abs(spec.q))):
        err = np.abs(J[c] - ref.J[c]).max()
        bound = n * (2.0 ** -24 + 2.0 ** -30) * unit + 2.0 ** -23 * np.abs(ref.J[c]).max()
        flush(f"{n} particles in one cell, J{'xyz'[c]}: max error {err:.3e}, bound {bound:.3e}, "
              f"rel err {rel_err(J[c], ref.J[c]):.2e}")
        assert err <= bound
    sim.sort()
    assert sim.check() == 0
    sim.close()


@pytest.mark.parametrize("nx,ny", [(32752, 16), (16, 32752)])
def test_largest_grid_extent(nx, ny):
    from paper_2501_14795_amd import Sim
    spec = pw.SpeciesSpec(-1.0, (1, 1), (0.3, 0.3, 0.3), (0.2, -0.2, 0.0))
    st = pw.species_state(nx, ny, 16, spec, 3)
    E, B = pw.random_fields(nx, ny, 0.05, 3)
    sim = Sim(nx, ny, DX, DY, DT, 16, [(spec.qm, spec.q, st)], E=E, B=B)
    ref = oracle_from_gpu(sim, [spec], DX, DY, DT)
    ref.push_deposit()
    sim.push_deposit()
    assert sim.check() == 0
    g = sim.state(0)
    pos, du = particle_errors(g, ref.species[0], nx, ny)
    e = rel_err(sim.field_arrays()["J"], ref.J)
    seam = int(((st["ix"] == nx - 1) & (g["ix"] == 0)).sum() + ((st["ix"] == 0) & (g["ix"] == nx - 1)).sum() +
               ((st["iy"] == ny - 1) & (g["iy"] == 0)).sum() + ((st["iy"] == 0) & (g["iy"] == ny - 1)).sum())
    flush(f"{nx} x {ny}: pos {pos:.2e} u {du:.2e} J {e:.2e}; {seam} particles crossed the periodic seam")
    assert seam > 0
    assert pos < 1e-5 and du < 1e-5 and e < 1e-5
    assert int(g["ix"].max()) < nx and int(g["iy"].max()) < ny and int(g["cell"].min()) >= 0
    sort_replay(sim, [spec], 16)
    sim.field_advance()
    assert sim.check() == 0
    sim.close()

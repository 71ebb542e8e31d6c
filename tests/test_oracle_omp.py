"""The OpenMP driver of the oracle (the benchmark's timed CPU baseline, the
paper's CPU implementation of Sec. 4.2.1: an OpenMP loop over tiles, a
private current per thread) against the serial oracle: the same canonical
sort bit for bit, the same step to FP64 round-off (the current is summed in
another order)."""
import numpy as np
import pytest

import pic_workloads as pw


def test_parallel_canonical_sort_equals_the_serial_one(ora):
    rng = np.random.default_rng(5)
    for T, nx, ny, n in ((8, 64, 32, 5000), (16, 64, 64, 20000), (4, 12, 8, 300), (8, 16, 8, 0), (1, 2, 1, 7)):
        ix = rng.integers(0, nx, n)
        iy = rng.integers(0, ny, n)
        a = ora.sort_canonical(nx, ny, T, ix, iy)
        b = ora.sort_canonical_omp(nx, ny, T, ix, iy)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    with pytest.raises(ValueError):
        ora.sort_canonical_omp(16, 16, 8, [16], [0])


def test_openmp_steps_equal_the_serial_oracle(ora):
    w = pw.WORKLOADS["uniform64"]
    st = pw.workload_state(w)[0]
    E, B = pw.random_fields(w.nx, w.ny, 0.05, 3)
    s = w.species[0]

    def species():
        return [ora.OracleSpecies(s.qm, s.q, st["ix"], st["iy"], st["x"], st["y"], st["ux"], st["uy"], st["uz"])]

    serial = ora.OracleSim(w.nx, w.ny, w.dx, w.dy, w.dt, species(), E.astype(np.float64), B.astype(np.float64))
    par = ora.OracleOmpSim(w.nx, w.ny, w.dx, w.dy, w.dt, species(), w.tile, E.astype(np.float64),
                           B.astype(np.float64))
    for _ in range(5):
        serial.step(T=w.tile)
        par.step(T=w.tile)
        for name in ("E", "B", "J"):
            a, b = getattr(serial, name), getattr(par, name)
            assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max(), name
        p, q = serial.species[0], par.species[0]
        assert np.array_equal(p.ix, q.ix) and np.array_equal(p.iy, q.iy)
        for name in ("x", "y", "ux", "uy", "uz"):
            assert np.abs(getattr(p, name) - getattr(q, name)).max() <= 1e-12, name
    assert ora.omp_threads() >= 1

"""pic_solve_gauss_noalloc, the allocation-free variant of pic_solve_gauss
(whose results test_gpu_gauss.py checks against the oracle's exact
projection), called through the C ABI.

Two calls in a row, the second on a smaller grid (the static scratch keeps
the first call's contents): each time twin simulations from the same state
are solved, one with a caller workspace (pic_solve_gauss), one in the
library's static scratch.  The node charge density both start from is
summed with FP64 atomics, so the two solves agree to round-off, not bit
for bit: E and B within 4 FP32 ulps of max|F| (the bound test_gpu_gauss.py
uses for the stored fields), both converged, iteration counts equal up to
the solver's convergence-check interval of 16.  A grid beyond the scratch's
capacity is refused with PIC_ESCRATCH and its fields are left as they
were."""
import numpy as np
import pytest

import pic_workloads as pw
from _parity import flush

pytestmark = pytest.mark.gpu

DX, DY, DT = 0.1, 0.12, 0.06


def _state(nx, ny, tile, seed):
    spec = pw.SpeciesSpec(-1.0, (3, 3), (0.05, 0.05, 0.05), (0.0, 0.0, 0.0))
    st = pw.species_state(nx, ny, tile, spec, seed)
    rng = np.random.default_rng(seed)
    st["x"] = rng.uniform(0.0, 1.0, st["x"].size).astype(np.float32)
    st["y"] = rng.uniform(0.0, 1.0, st["y"].size).astype(np.float32)
    st["x"][st["x"] >= 1.0] = 0.0
    st["y"][st["y"] >= 1.0] = 0.0
    E, B = pw.random_fields(nx, ny, 0.2, seed)
    B[0] += rng.normal(0, 0.05, (ny, nx)).astype(np.float32)
    return spec, st, E, B


def test_noalloc_equals_the_workspace_variant():
    from paper_2501_14795_amd import Sim, _lib
    for nx, ny, seed in ((256, 192, 5), (64, 48, 6)):
        spec, st, E, B = _state(nx, ny, 16, seed)
        a = Sim(nx, ny, DX, DY, DT, 16, [(spec.qm, spec.q, st)], E=E, B=B)
        b = Sim(nx, ny, DX, DY, DT, 16, [(spec.qm, spec.q, st)], E=E, B=B)
        oa = a.solve_gauss()
        b.stream.synchronize()
        ob = _lib.pic_solve_gauss_noalloc(b.handle, 0.0, 0, b.s)
        fa, fb = a.field_arrays(), b.field_arrays()
        flush(f"{nx}x{ny}: iterations {list(oa.iterations)} / {list(ob.iterations)}, residuals "
              f"{list(oa.residual)} / {list(ob.residual)}")
        for k in range(2):
            assert abs(oa.iterations[k] - ob.iterations[k]) <= 16 and oa.iterations[k] > 0
            assert oa.residual[k] <= 1e-12 and ob.residual[k] <= 1e-12
        for k in ("E", "B"):
            scale = np.abs(fa[k]).max()
            diff = np.abs(fa[k].astype(np.float64) - fb[k]).max()
            flush(f"{nx}x{ny}: {k} differs by {diff:.2e} = {diff / scale:.2e} of max|{k}|")
            assert diff <= 4 * 2.0 ** -24 * scale, k
        assert not np.array_equal(fb["E"], E)   # the solve changed the fields
        assert a.check() == 0 and b.check() == 0
        a.close()
        b.close()


def test_noalloc_refuses_grids_beyond_its_scratch():
    from paper_2501_14795_amd import Sim, _lib
    nx, ny = 1024, 1040   # 1,064,960 cells > PIC_GAUSS_NOALLOC_MAX_CELLS
    assert nx * ny > _lib.PIC_GAUSS_NOALLOC_MAX_CELLS
    empty = {k: np.zeros(0, np.int32 if k in ("ix", "iy") else np.float32)
             for k in ("ix", "iy", "x", "y", "ux", "uy", "uz")}
    E, B = pw.random_fields(nx, ny, 0.1, 7)
    sim = Sim(nx, ny, DX, DY, DT, 16, [(-1.0, -1.0, empty)], E=E, B=B)
    sim.stream.synchronize()
    with pytest.raises(_lib.PicError) as e:
        _lib.pic_solve_gauss_noalloc(sim.handle, 0.0, 0, sim.s)
    assert e.value.code == _lib.PIC_ESCRATCH
    f = sim.field_arrays()
    assert np.array_equal(f["E"], E) and np.array_equal(f["B"], B)
    sim.close()

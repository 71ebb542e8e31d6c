"""Valid initial fields (pic_solve_gauss; Sec. 3.2, Eqs. 17-18) on the GPU
against the oracle's exact projection.

The GPU solves the two periodic Poisson problems by FP64 conjugate gradients
and stores FP32 fields; the oracle solves them exactly by FFT.  From the same
state (random E and B with a divergence, a non-uniform particle charge):
E and B within 1e-6 of max|F| of the oracle's; afterwards the Gauss and div B
residuals of pic_diag are at the FP32 rounding of the stored fields,
4 * 2^-24 * max|F| / min(dx, dy).  The cold Langmuir start: from E = 0 the
solve reproduces the one-dimensional Gauss construction, and the run keeps
Gauss's law.  Errors: short scratch, an iteration cap that stops the solve
early."""
import os
import sys

import numpy as np
import pytest

import oracle
import pic_workloads as pw
from _parity import flush, rel_err

pytestmark = pytest.mark.gpu

DX, DY, DT = 0.1, 0.12, 0.06


def _lib():
    from paper_2501_14795_amd import _lib
    return _lib


def _jittered(nx, ny, tile, seed):
    """A 3 x 3 ppc lattice with the offsets jittered inside each cell:
    non-uniform charge, still grouped by tile."""
    spec = pw.SpeciesSpec(-1.0, (3, 3), (0.05, 0.05, 0.05), (0.0, 0.0, 0.0))
    st = pw.species_state(nx, ny, tile, spec, seed)
    rng = np.random.default_rng(seed)
    st["x"] = rng.uniform(0.0, 1.0, st["x"].size).astype(np.float32)
    st["y"] = rng.uniform(0.0, 1.0, st["y"].size).astype(np.float32)
    st["x"][st["x"] >= 1.0] = 0.0
    st["y"][st["y"] >= 1.0] = 0.0
    return spec, st


def test_solve_gauss_matches_oracle():
    from paper_2501_14795_amd import Sim
    L = _lib()
    nx, ny, tile = 64, 48, 16
    spec, st = _jittered(nx, ny, tile, 3)
    E, B = pw.random_fields(nx, ny, 0.2, 3)
    B[0] += np.random.default_rng(4).normal(0, 0.05, (ny, nx)).astype(np.float32)
    sim = Sim(nx, ny, DX, DY, DT, tile, [(spec.qm, spec.q, st)], E=E, B=B)
    before = sim.diag(L.PIC_DIAG_GAUSS)
    g = sim.state(0)
    rho = oracle.rho(nx, ny, spec.q, g["ix"], g["iy"], g["x"], g["y"])
    f0 = sim.field_arrays()
    Eo, Bo = f0["E"].astype(np.float64), f0["B"].astype(np.float64)
    oracle.solve_gauss(nx, ny, DX, DY, Eo, Bo, rho)
    out = sim.solve_gauss()
    f = sim.field_arrays()
    eE, eB = rel_err(f["E"], Eo), rel_err(f["B"], Bo)
    after = sim.diag(L.PIC_DIAG_GAUSS)
    bound_e = 4 * 2.0 ** -24 * np.abs(f["E"]).max() / min(DX, DY)
    bound_b = 4 * 2.0 ** -24 * np.abs(f["B"]).max() / min(DX, DY)
    flush(f"iterations {list(out.iterations)}, residuals {list(out.residual)}; E {eE:.2e} B {eB:.2e} vs oracle; "
          f"gauss {before.gauss_max:.2e} -> {after.gauss_max:.2e} (bound {bound_e:.2e}), "
          f"div B {before.divb_max:.2e} -> {after.divb_max:.2e} (bound {bound_b:.2e})")
    assert eE <= 1e-6 and eB <= 1e-6
    assert after.gauss_max <= bound_e and after.divb_max <= bound_b
    assert before.gauss_max > 1e3 * bound_e and before.divb_max > 1e3 * bound_b
    assert out.residual[0] <= 1e-12 and out.residual[1] <= 1e-12
    assert np.array_equal(f["E"][2], f0["E"][2]) and np.array_equal(f["B"][2], f0["B"][2])
    sim.close()


def test_solve_gauss_langmuir_start():
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    from langmuir_fixture import DT as LDT, DX as LDX, langmuir_state
    from paper_2501_14795_amd import Sim
    L = _lib()
    nx, ny, tile = 256, 16, 16
    spec, st, E_ref = langmuir_state(nx, ny, tile)
    sim = Sim(nx, ny, LDX, LDX, LDT, tile, [(spec.qm, spec.q, st)])
    out = sim.solve_gauss()
    E = sim.field_arrays()["E"]
    e = rel_err(E, E_ref)
    g0 = sim.diag(L.PIC_DIAG_GAUSS).gauss_max
    for _ in range(50):
        sim.step()
    g = sim.diag(L.PIC_DIAG_GAUSS).gauss_max
    # at the start: the FP32 rounding of the stored field; after n steps also
    # the current's per-step continuity error (about 1e-7 of max|rho|), as a
    # random walk: 8 sqrt(n) (2^-23 max|E| / dx + 1e-7 max|rho|)
    bound0 = 8 * 2.0 ** -24 * np.abs(E_ref).max() / LDX
    rho_max = abs(spec.q) * 32 * 1.01
    bound = 8 * np.sqrt(50) * (2.0 ** -23 * np.abs(E_ref).max() / LDX + 1e-7 * rho_max)
    flush(f"Langmuir start from E = 0: {list(out.iterations)} iterations, Ex vs prefix sum {e:.2e}; "
          f"gauss {g0:.2e} (bound {bound0:.2e}) -> {g:.2e} after 50 steps (bound {bound:.2e})")
    assert e <= 1e-6
    assert g0 <= bound0 and g <= bound
    assert sim.check() == 0
    sim.close()


def test_solve_gauss_errors():
    import torch
    from paper_2501_14795_amd import PicError, Sim
    L = _lib()
    nx, ny, tile = 32, 32, 16
    spec, st = _jittered(nx, ny, tile, 5)
    sim = Sim(nx, ny, DX, DY, DT, tile, [(spec.qm, spec.q, st)])
    small = torch.empty(1 << 12, dtype=torch.uint8, device="cuda")
    with pytest.raises(PicError) as e:
        L.pic_solve_gauss(sim.handle, small.data_ptr(), small.numel(), 0.0, 0, sim.s)
    assert e.value.code == L.PIC_EINVAL
    with pytest.raises(PicError) as e:       # one iteration cannot reach 1e-12
        sim.solve_gauss(max_iter=1)
    assert e.value.code == L.PIC_ENOCONV
    out = sim.solve_gauss()                  # a full solve still works afterwards
    assert out.residual[0] <= 1e-12
    sim.close()

"""GPU diagnostics of Gauss's law and div B, and state I/O (checkpoint /
resume) through the C ABI.

* PIC_DIAG_GAUSS against the oracle's node charge, div E and div B evaluated
  on the GPU's own FP32 state (both FP64; only the order of the charge sums
  differs).
* The residuals stay at their initial values over a run: the deposit is
  charge conserving (Eq. 12) and the Yee curls are divergence free.
* pic_get_state / pic_set_state: a round trip is bit-exact, a run resumed from
  a checkpoint equals the uninterrupted run bit for bit (fixed-point current),
  and particles not grouped by tile are rejected.
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle
import pic_workloads as pw
from _parity import flush, species_states

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
from langmuir_fixture import DT, DX, langmuir_state  # noqa: E402

pytestmark = pytest.mark.gpu


def _uniform(E=None, B=None, seed=1):
    from paper_2501_14795_amd import Sim
    w = pw.WORKLOADS["uniform64"]
    st = species_states(w.nx, w.ny, w.tile, w.species, seed)
    spec = w.species[0]
    return Sim(w.nx, w.ny, w.dx, w.dy, w.dt, w.tile, [(spec.qm, spec.q, st[0])], E=E, B=B), w


def _oracle_residuals(sim, w):
    f = sim.field_arrays()
    spec = w.species[0]
    g = sim.state(0)
    rho = oracle.rho(w.nx, w.ny, spec.q, g["ix"], g["iy"], g["x"], g["y"])
    gauss = oracle.div_e(w.nx, w.ny, w.dx, w.dy, f["E"].astype(np.float64)) - (rho - rho.mean())
    divb = oracle.div_b(w.nx, w.ny, w.dx, w.dy, f["B"].astype(np.float64))
    return np.abs(gauss).max(), np.abs(divb).max(), np.abs(rho).max()


def test_gauss_diag_matches_oracle():
    from paper_2501_14795_amd import _lib
    E, B = pw.random_fields(64, 64, 0.1, 21)
    sim, w = _uniform(E, B)
    for step in range(3):
        d = sim.diag(_lib.PIC_DIAG_GAUSS)
        g, b, _ = _oracle_residuals(sim, w)
        flush(f"step {step}: gauss {d.gauss_max:.6e} (oracle {g:.6e}), div B {d.divb_max:.6e} (oracle {b:.6e})")
        assert g > 1e-3 and b > 1e-3
        assert abs(d.gauss_max - g) <= 1e-12 * g
        assert abs(d.divb_max - b) <= 1e-12 * b
        sim.step()
    # GAUSS alone leaves no rho snapshot behind
    with pytest.raises(_lib.PicError):
        sim.diag(_lib.PIC_DIAG_CONTINUITY)
    assert sim.check() == 0
    sim.close()


def test_gauss_and_divb_preserved_thermal():
    """Thermal plasma from E = B = 0 and an exactly uniform lattice charge:
    both residuals start at round-off and stay there while the fields grow
    from the noise.  Bounds: FP32 E and B carry relative rounding 2^-24 per
    update, so after n steps the differences of neighbours err by about
    sqrt(n) * 2^-23 * max|F| / d; the FP32 current adds its own continuity
    error, dt * 2 ulp(J) / dx < 1e-7 max|rho| per step."""
    from paper_2501_14795_amd import _lib
    sim, w = _uniform()
    d0 = sim.diag(_lib.PIC_DIAG_GAUSS)
    _, _, rho_max = _oracle_residuals(sim, w)
    n = 40
    for _ in range(n):
        sim.step()
    d = sim.diag(_lib.PIC_DIAG_GAUSS)
    f = sim.field_arrays()
    emax, bmax = np.abs(f["E"][:2]).max(), np.abs(f["B"][:2]).max()
    bound_e = 8 * math.sqrt(n) * (2.0 ** -23 * emax / w.dx + 1e-7 * rho_max)
    bound_b = 8 * math.sqrt(n) * 2.0 ** -23 * bmax / w.dx
    flush(f"initial gauss {d0.gauss_max:.2e} div B {d0.divb_max:.2e}; after {n} steps gauss {d.gauss_max:.2e} "
          f"(bound {bound_e:.2e}, max|E| {emax:.2e}) div B {d.divb_max:.2e} (bound {bound_b:.2e}, "
          f"max|B| {bmax:.2e})")
    assert d0.gauss_max < 1e-9 * rho_max and d0.divb_max == 0.0
    assert emax > 1e-4 and bmax > 1e-6            # the fields did grow
    assert d.gauss_max <= bound_e
    assert d.divb_max <= bound_b
    sim.close()


def test_gauss_preserved_langmuir():
    """Langmuir start with Ex from the discrete Gauss law: the residual starts at
    the FP32 rounding of Ex and grows over 300 steps only as the round-off
    walk of the thermal case (FP32 E updates plus the per-step continuity
    error of the current, each contribution rounded to 2^-23 of the largest
    one), far below the 1e-3 charge perturbation a non-conserving deposit
    would leave behind; B stays exactly zero."""
    from paper_2501_14795_amd import Sim, _lib
    nx, ny = 256, 16
    spec, st, E = langmuir_state(nx, ny, 16)
    sim = Sim(nx, ny, DX, DX, DT, 16, [(spec.qm, spec.q, st)], E=E.astype(np.float32))
    d0 = sim.diag(_lib.PIC_DIAG_GAUSS)
    worst = 0.0
    for n in range(1, 301):
        sim.step()
        if n % 50 == 0:
            d = sim.diag(_lib.PIC_DIAG_GAUSS)
            worst = max(worst, d.gauss_max)
            assert d.divb_max == 0.0
    emax = float(np.abs(E[0]).max())
    flush(f"langmuir {nx}x{ny}: gauss initial {d0.gauss_max:.2e}, worst over 300 steps {worst:.2e}, "
          f"max|Ex| {emax:.2e}")
    rho_max = abs(spec.q) * spec.n_ppc * (1 + 1e-3)
    assert d0.gauss_max < 4 * 2.0 ** -24 * emax / DX + 1e-12
    assert worst <= 8 * math.sqrt(300) * (2.0 ** -23 * emax / DX + 1e-7 * rho_max)
    sim.close()


def test_state_round_trip_and_resume():
    from paper_2501_14795_amd import _lib
    E, B = pw.random_fields(64, 64, 0.05, 5)
    sim, w = _uniform(E, B)
    for _ in range(3):
        sim.step()
    ck = sim.get_state()
    # round trip through the C ABI is bit-exact
    sim.set_state(ck)
    again = sim.get_state()
    assert np.array_equal(again["fields"], ck["fields"])
    for a in ck["species"][0]:
        assert np.array_equal(again["species"][0][a], ck["species"][0][a]), a
    off_ck = sim.tile_offsets(0)
    for _ in range(4):
        sim.step()
    ref = sim.get_state()
    # resume the same simulation from the checkpoint
    sim.set_state(ck)
    assert np.array_equal(sim.tile_offsets(0), off_ck)
    for _ in range(4):
        sim.step()
    out = sim.get_state()
    assert np.array_equal(out["fields"], ref["fields"])
    for a in ref["species"][0]:
        assert np.array_equal(out["species"][0][a], ref["species"][0][a]), a
    # and a fresh simulation started from other particles (same counts)
    sim2, _ = _uniform(seed=9)
    sim2.set_state(ck)
    for _ in range(4):
        sim2.step()
    out2 = sim2.get_state()
    assert np.array_equal(out2["fields"], ref["fields"])
    for a in ref["species"][0]:
        assert np.array_equal(out2["species"][0][a], ref["species"][0][a]), a
    assert sim.check() == 0 and sim2.check() == 0
    # particles not grouped by tile: grouped on load (stable), as the oracle does
    rev = {k: v[::-1].copy() for k, v in ck["species"][0].items()}
    sim2.set_state({"fields": ck["fields"], "species": [rev]})
    ix, iy = rev["cell"] & 0xFFFF, rev["cell"] >> 16
    _, src = oracle.sort_stable_by_tile(sim2.nx, sim2.ny, 16, ix, iy)
    got = sim2.get_state()["species"][0]
    for a in rev:
        assert np.array_equal(got[a], rev[a][src]), a
    # a cell outside the grid: rejected
    bad = {k: v.copy() for k, v in ck["species"][0].items()}
    bad["cell"][7] = sim2.nx + 3
    with pytest.raises(_lib.PicError) as e:
        sim2.set_state({"fields": ck["fields"], "species": [bad]})
    assert e.value.code == _lib.PIC_EORDER
    sim2.set_state(ck)
    sim2.step()
    assert sim2.check() == 0
    sim.close()
    sim2.close()

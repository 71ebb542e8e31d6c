"""Cold Langmuir oscillation: initial state and the oracle's reference history.

Initial state: a cold electron lattice, 32 per cell (8 x 4), displaced along x
by xi(X) = -(A/k) sin(k X) (density n0 (1 + A cos kX), A = 1e-3, k the
fundamental mode of an nx-cell box), regrouped by tile; Ex from the discrete
Gauss law (Eq. 17) with a neutralising ion background, computed from the
oracle's node charge; B = 0, u = 0.  Every row of cells is identical, so the
run is one-dimensional and its energies scale with ny.

Run as a script, it advances the 1024 x 16 case with the oracle only and writes
langmuir_1024x16_oracle.txt (step, total energy, field energy, kinetic
energy, Ex mode amplitude of row 0) every 5 steps up to step 1500 and every
250 steps up to step 5000.
"""
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import pic_workloads as pw  # noqa: E402

DX = 0.1
DT = 0.07
AMP = 1e-3
FIXTURE = os.path.join(HERE, "langmuir_1024x16_oracle.txt")


def langmuir_state(nx, ny, tile, ppc=(8, 4), amp=AMP):
    spec = pw.SpeciesSpec(-1.0, ppc, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    st = pw.species_state(nx, ny, tile, spec, 5)
    k = 2 * math.pi / nx                               # per cell
    X0 = st["ix"] + st["x"].astype(np.float64)
    X = (X0 - (amp / k) * np.sin(k * X0)) % nx
    ix = np.floor(X).astype(np.int32)
    x = (X - ix).astype(np.float32)
    up = x >= 1.0
    x[up] = 0.0
    ix[up] += 1
    ix %= nx
    tile_id = (st["iy"] // tile) * (nx // tile) + ix // tile
    order = np.argsort(tile_id, kind="stable")
    out = {"ix": ix[order], "iy": st["iy"][order], "x": x[order], "y": st["y"][order],
           "ux": st["ux"][order], "uy": st["uy"][order], "uz": st["uz"][order]}
    # Gauss: (Ex[i] - Ex[i-1]) / dx = rho[i] - <rho>, Ex zero-mean (Ex at i+1/2)
    rho = oracle.rho(nx, ny, spec.q, out["ix"], out["iy"], out["x"], out["y"])
    r = rho.mean(axis=0) - rho.mean()
    ex = np.cumsum(r) * DX
    ex -= ex.mean()
    E = np.zeros((3, ny, nx))
    E[0] = ex[None, :]
    return spec, out, E


def mode_weights(nx):
    return np.sin(2 * math.pi / nx * (np.arange(nx) + 0.5))


def read_fixture():
    rows = np.loadtxt(FIXTURE, comments="#")
    return {int(r[0]): r[1:] for r in rows}


def recorded(n):
    return (n <= 1500 and n % 5 == 0) or n % 250 == 0


def main(steps=5000):
    nx, ny = 1024, 16
    spec, st, E = langmuir_state(nx, ny, 16)
    osp = oracle.OracleSpecies(spec.qm, spec.q, st["ix"], st["iy"], st["x"], st["y"], st["ux"], st["uy"],
                               st["uz"])
    ora = oracle.OracleSim(nx, ny, DX, DX, DT, [osp], E.astype(np.float32).astype(np.float64))
    w = mode_weights(nx)
    lines = ["# FP64 oracle, cold Langmuir oscillation, 1024 x 16 cells, 32 ppc, A = 1e-3, dx = 0.1, dt = 0.07",
             "# written by tests/golden/langmuir_fixture.py (oracle only)",
             "# step  U_total  U_E  U_K  Ex_mode(row 0)"]
    for n in range(1, steps + 1):
        ora.step(T=16)
        if recorded(n):
            ue, ub, uk = ora.energies()
            lines.append(f"{n} {ue + ub + uk[0]:.12e} {ue:.12e} {uk[0]:.12e} {ora.E[0, 0] @ w:.12e}")
            print(lines[-1], flush=True)
    with open(FIXTURE, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()

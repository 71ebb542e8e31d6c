"""Seeded synthetic workloads shared by the GPU path's callers and by the oracle.

This module holds no arithmetic of the PIC method: it only lays out the initial
particle state (regular sub-lattice positions inside every cell, Gaussian
momenta from a seeded Philox generator) and names the workloads.  Both sides
receive the same FP32 arrays; the oracle widens them to FP64.

Particle order.  Particles are emitted tile by tile (tiles of T x T cells,
row-major), and inside a tile sub-lattice slot by slot: all cells' slot 0 (in
row-major cell order), then all cells' slot 1, and so on.  Consecutive
particles therefore sit in different cells, which is the array order a tiled
particle kernel wants; the physics does not depend on it.

The paper's own decks (cold / warm uniform plasma, Weibel; Sec. 5.1) are not
available; the workloads below are synthetic stand-ins with the same structure
(uniform periodic plasma, Maxwellian momenta, counter-streaming beams).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Tuple

import numpy as np


@dataclasses.dataclass
class SpeciesSpec:
    qm: float = -1.0                 # charge-to-mass ratio (electrons: -1)
    ppc: Tuple[int, int] = (4, 4)    # sub-lattice per cell (x, y)
    u_th: Tuple[float, float, float] = (0.1, 0.1, 0.1)
    u_fl: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    n0: float = 1.0                  # density in units of the normalising density

    @property
    def n_ppc(self) -> int:
        return self.ppc[0] * self.ppc[1]

    @property
    def q(self) -> float:
        """Charge density carried by one macro-particle (sign of qm, n0/ppc)."""
        return float(np.sign(self.qm)) * self.n0 / self.n_ppc


@dataclasses.dataclass
class Workload:
    name: str
    nx: int
    ny: int
    dx: float
    dy: float
    dt: float
    tile: int
    steps: int
    seed: int
    species: List[SpeciesSpec]
    description: str = ""

    @property
    def n_particles(self) -> int:
        return sum(self.nx * self.ny * s.n_ppc for s in self.species)


WORKLOADS = {
    "uniform64": Workload(
        "uniform64", 64, 64, 0.1, 0.1, 0.07, 16, 100, 1,
        [SpeciesSpec(-1.0, (4, 4), (0.1, 0.1, 0.1), (0.0, 0.0, 0.0))],
        "64x64 cells, 16 ppc thermal electrons u_th=0.1, periodic, tile 16"),
    "weibel512": Workload(
        "weibel512", 512, 512, 0.1, 0.1, 0.07, 16, 500, 2,
        [SpeciesSpec(-1.0, (8, 8), (0.1, 0.1, 0.1), (0.0, 0.0, 0.6)),
         SpeciesSpec(-1.0, (8, 8), (0.1, 0.1, 0.1), (0.0, 0.0, -0.6))],
        "512x512 cells, two electron beams u_fl=+-0.6 along z, 64 ppc each"),
    "warm2048": Workload(
        "warm2048", 2048, 2048, 0.1, 0.1, 0.07, 32, 200, 3,
        [SpeciesSpec(-1.0, (4, 4), (0.05, 0.05, 0.05), (0.2, 0.0, 0.0))],
        "2048x2048 cells, 16 ppc warm electrons u_th=0.05 drifting u_x=0.2, tile 32"),
    "langmuir1024": Workload(
        "langmuir1024", 1024, 1024, 0.1, 0.1, 0.07, 16, 10000, 5,
        [SpeciesSpec(-1.0, (8, 4), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0))],
        "1024x1024 cells, 32 ppc cold electrons (perturbation applied by caller)"),
}


def species_state(nx: int, ny: int, tile: int, spec: SpeciesSpec, seed: int,
                  species_index: int = 0, cell_box: Optional[Tuple[int, int, int, int]] = None):
    """Initial particles of one species, in tile order (see module docstring).

    Returns a dict of numpy arrays: ix, iy (int32), x, y, ux, uy, uz (float32).
    ``cell_box = (x0, x1, y0, y1)`` restricts the loading to those cells
    (used to build ragged / empty-tile cases); particles outside are dropped.
    """
    T = tile
    if nx % T or ny % T:
        raise ValueError("grid must be a whole number of tiles")
    ntx, nty = nx // T, ny // T
    px, py = spec.ppc
    # axes: (tile_y, tile_x, slot_y, slot_x, cell_y, cell_x)
    ty = np.arange(nty, dtype=np.int32)[:, None, None, None, None, None]
    tx = np.arange(ntx, dtype=np.int32)[None, :, None, None, None, None]
    sb = np.arange(py, dtype=np.int32)[None, None, :, None, None, None]
    sa = np.arange(px, dtype=np.int32)[None, None, None, :, None, None]
    cy = np.arange(T, dtype=np.int32)[None, None, None, None, :, None]
    cx = np.arange(T, dtype=np.int32)[None, None, None, None, None, :]
    shape = (nty, ntx, py, px, T, T)
    ix = np.broadcast_to(tx * T + cx, shape).reshape(-1)
    iy = np.broadcast_to(ty * T + cy, shape).reshape(-1)
    x = np.broadcast_to(((sa + 0.5) / px).astype(np.float32), shape).reshape(-1)
    y = np.broadcast_to(((sb + 0.5) / py).astype(np.float32), shape).reshape(-1)
    if cell_box is not None:
        x0, x1, y0, y1 = cell_box
        keep = (ix >= x0) & (ix < x1) & (iy >= y0) & (iy < y1)
        ix, iy, x, y = ix[keep], iy[keep], x[keep], y[keep]
    n = ix.size
    rng = np.random.Generator(np.random.Philox(np.random.SeedSequence([seed, species_index])))
    u = []
    for k in range(3):
        if spec.u_th[k] != 0.0:
            v = spec.u_fl[k] + spec.u_th[k] * rng.standard_normal(n)
        else:
            v = np.full(n, spec.u_fl[k])
        u.append(v.astype(np.float32))
    return {
        "ix": np.ascontiguousarray(ix, dtype=np.int32),
        "iy": np.ascontiguousarray(iy, dtype=np.int32),
        "x": np.ascontiguousarray(x, dtype=np.float32),
        "y": np.ascontiguousarray(y, dtype=np.float32),
        "ux": u[0], "uy": u[1], "uz": u[2],
    }


def workload_state(w: Workload, tile: Optional[int] = None):
    """Initial particles of every species of a workload (list of dicts)."""
    T = w.tile if tile is None else tile
    return [species_state(w.nx, w.ny, T, s, w.seed, k) for k, s in enumerate(w.species)]


def random_fields(nx: int, ny: int, amp: float, seed: int):
    """Smooth-ish random E and B (3, ny, nx) float32 planes for parity tests:
    a few random Fourier modes per component, so the fields are resolved on
    the grid.  Amplitude ``amp``."""
    rng = np.random.Generator(np.random.Philox(np.random.SeedSequence([seed, 1000])))
    X = np.arange(nx)[None, :]
    Y = np.arange(ny)[:, None]
    out = []
    for _ in range(2):
        comps = []
        for _c in range(3):
            f = np.zeros((ny, nx))
            for _m in range(3):
                kx = rng.integers(0, 4)
                ky = rng.integers(0, 4)
                ph = rng.uniform(0, 2 * np.pi)
                a = rng.uniform(-1, 1)
                f += a * np.cos(2 * np.pi * (kx * X / nx + ky * Y / ny) + ph)
            comps.append(amp * f / 3.0)
        out.append(np.stack(comps).astype(np.float32))
    return out[0], out[1]


PPC_LATTICE = {8: (4, 2), 16: (4, 4), 32: (8, 4), 64: (8, 8)}


def batched_members(n_sims: int = 256, seed: int = 4, sizes=(32, 64, 96, 128, 160, 192, 224, 256),
                    ppcs=(8, 16, 32, 64), dx: float = 0.1, dt: float = 0.07):
    """Specifications of many independent small simulations (the batched
    workload): nx and ny independently uniform on `sizes`, particles per cell
    uniform on `ppcs`, u_th ~ U[0.01, 0.2] isotropic, drift zero with
    probability 1/2 else each component ~ U[-0.3, 0.3].  One electron species
    each.  Returns a list of dicts (nx, ny, dx, dy, dt, spec, seed)."""
    rng = np.random.Generator(np.random.Philox(np.random.SeedSequence([seed, 7777])))
    out = []
    for k in range(n_sims):
        nx = int(rng.choice(sizes))
        ny = int(rng.choice(sizes))
        ppc = int(rng.choice(ppcs))
        u_th = float(rng.uniform(0.01, 0.2))
        drift = (0.0, 0.0, 0.0) if rng.random() < 0.5 else tuple(float(v) for v in rng.uniform(-0.3, 0.3, 3))
        spec = SpeciesSpec(-1.0, PPC_LATTICE[ppc], (u_th,) * 3, drift)
        out.append({"nx": nx, "ny": ny, "dx": dx, "dy": dx, "dt": dt, "spec": spec, "seed": seed * 100000 + k})
    return out

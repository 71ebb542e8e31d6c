"""The method's edge cases placed by hand and pushed through the HIP kernel,
checked against the oracle from the GPU's own state.

E = B = 0, so every particle moves on a straight line with its loaded
momentum, and the motions below are reached exactly:
  * corner hits: a motion that crosses an x face and a y face at the same
    instant (x = y and ux = uy, in all four diagonal directions) -- the
    split's tie, a zero-length middle piece;
  * exact face landings: x + dX rounding to exactly 1.0 in FP32 (and y + dY),
    and x + dX = 0 from inside the cell -- 129 starting offsets one ulp apart
    around 1 - dX, so that several of them land on the face whatever the last
    bit of the kernel's dX;
  * zero motion (ux = uy = 0, uz != 0: only Jz);
  * x = 0 (and y = 0) with a backward step smaller than half an ulp of 1.0:
    x + 1 rounds to 1.0 in FP32, which the kernel stores as x = 0 of the old
    cell (the offset rule); the oracle keeps x = 1 - 7e-9 of the cell below;
  * x = nextafter(1, 0) (and y) with a tiny forward step;
  * crossings from every tile into each of its eight neighbour tiles, so the
    tiles of the grid's edge cross the periodic seam.
Checks: particles within 1e-5 cells / 1e-5 max|u| slot by slot, J within
1e-5 max|J| node by node, every offset in [0, 1) after the step, and the
sort bit-exact against the oracle's canonical sort of the GPU's cells.
"""
import numpy as np
import pytest

from _parity import flush, oracle_from_gpu, particle_errors, rel_err, sort_replay

pytestmark = pytest.mark.gpu

DX = DY = 0.1
DT = 0.07
TOL = 1e-5


class _Spec:
    qm = -1.0
    q = -1.0 / 16


def _dX(u):
    """Displacement in cells of momentum u = (ux, uy, uz) (Eq. 11), FP64."""
    g = np.sqrt(1.0 + (np.asarray(u, np.float64) ** 2).sum())
    return u[0] / g * DT / DX, u[1] / g * DT / DY


def _edge_particles(T):
    n_t = 3
    nx = ny = n_t * T
    P = {k: [] for k in ("ix", "iy", "x", "y", "ux", "uy", "uz")}

    def add(ix, iy, x, y, u):
        P["ix"].append(ix % nx)
        P["iy"].append(iy % ny)
        P["x"].append(np.float32(x))
        P["y"].append(np.float32(y))
        for k, v in zip(("ux", "uy", "uz"), u):
            P[k].append(np.float32(v))

    c = T + T // 2   # a cell in the middle tile
    # corner hits, all four diagonals
    for sx in (-1, 1):
        for sy in (-1, 1):
            x0 = 0.75 if sx > 0 else 0.25
            y0 = 0.75 if sy > 0 else 0.25
            add(c, c, x0, y0, (0.6 * sx, 0.6 * sy, 0.1))
    # landings on x = 1, y = 1 (forward) and x = 0, y = 0 (from inside)
    f32 = np.float32
    for axis in (0, 1):
        for fwd in (True, False):
            u = [0.0, 0.0, 0.05]
            u[axis] = 0.45 if fwd else -0.45
            u = [f32(v) for v in u]
            d = _dX(np.array(u, np.float64))[axis]
            start = f32(1.0 - d) if fwd else f32(-d)
            xs = [start]
            lo = hi = start
            for _ in range(64):
                lo = np.nextafter(lo, f32(0))
                hi = np.nextafter(hi, f32(1))
                xs += [lo, hi]
            for v in xs:
                if axis == 0:
                    add(c, c + 1, v, 0.5, u)
                else:
                    add(c + 1, c, 0.5, v, u)
    # zero motion
    add(c - 1, c - 1, 0.3, 0.6, (0.0, 0.0, 0.2))
    add(c - 1, c - 1, 0.0, 0.0, (0.0, 0.0, -0.2))
    # x = 0 / y = 0 with a backward step below half an ulp of 1.0
    add(c, c - 2, 0.0, 0.4, (-1e-8, 0.0, 0.0))
    add(c, c - 2, 0.4, 0.0, (0.0, -1e-8, 0.0))
    add(c, c - 2, 0.0, 0.0, (-1e-8, -1e-8, 0.0))
    # the largest offset below 1 with a tiny forward step
    below1 = np.nextafter(f32(1.0), f32(0.0))
    add(c + 2, c, below1, 0.5, (1e-8, 0.0, 0.0))
    add(c + 2, c, 0.5, below1, (0.0, 1e-8, 0.0))
    add(c + 2, c, below1, below1, (1e-8, 1e-8, 0.0))
    # every tile into each of its eight neighbours (the edge tiles across the seam)
    for ty in range(n_t):
        for tx in range(n_t):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if dx == 0 and dy == 0:
                        continue
                    lx = T - 1 if dx > 0 else (0 if dx < 0 else T // 2)
                    ly = T - 1 if dy > 0 else (0 if dy < 0 else T // 3)
                    x0 = 0.9 if dx > 0 else (0.1 if dx < 0 else 0.5)
                    y0 = 0.85 if dy > 0 else (0.15 if dy < 0 else 0.5)
                    add(tx * T + lx, ty * T + ly, x0, y0, (0.35 * dx, 0.3 * dy, -0.05))
    st = {k: np.array(v, np.int32 if k in ("ix", "iy") else np.float32) for k, v in P.items()}
    return nx, ny, st


@pytest.mark.parametrize("tile,esirkepov", [(8, False), (16, False), (32, False), (16, True)])
def test_edge_cases_against_the_oracle(tile, esirkepov):
    from paper_2501_14795_amd import Sim
    nx, ny, st = _edge_particles(tile)
    spec = _Spec()
    sim = Sim(nx, ny, DX, DY, DT, tile, [(spec.qm, spec.q, st)], esirkepov=esirkepov)
    flush(f"[edges T={tile} esirkepov={esirkepov}] {st['ix'].size} particles on {nx}x{ny}")
    for step in range(2):
        ref = oracle_from_gpu(sim, [spec], DX, DY, DT)
        ref.esirkepov = esirkepov
        ref.push_deposit()
        sim.push_deposit()
        assert sim.check() == 0
        g = sim.state(0)
        assert (g["x"] >= 0).all() and (g["x"] < 1).all() and (g["y"] >= 0).all() and (g["y"] < 1).all()
        pos, du = particle_errors(g, ref.species[0], nx, ny)
        J = sim.field_arrays()["J"]
        ej = rel_err(J, ref.J)
        flush(f"[edges T={tile}] step {step}: pos {pos:.2e} u {du:.2e} J {ej:.2e}")
        assert pos < TOL and du < TOL and ej < TOL
        if step == 0:
            # the forward landings (momentum still the loaded one: E = B = 0)
            # include offsets that reached the next cell's face exactly
            f = np.float32
            on_x = (g["ux"] == f(0.45)) & (g["uy"] == 0) & (g["uz"] == f(0.05))
            on_y = (g["uy"] == f(0.45)) & (g["ux"] == 0) & (g["uz"] == f(0.05))
            assert on_x.sum() == 129 and on_y.sum() == 129
            assert (g["x"][on_x] == 0).sum() >= 1 and (g["y"][on_y] == 0).sum() >= 1
        sort_replay(sim, [spec], tile)
        sim.field_advance()
    assert sim.check() == 0
    sim.close()

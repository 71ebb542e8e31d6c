"""Shared helpers of the GPU-vs-oracle parity tests."""
from __future__ import annotations

import numpy as np

import oracle
import pic_workloads as pw

PARTICLE_ARRAYS = ("cell", "x", "y", "ux", "uy", "uz")


def flush(msg):
    print(msg, flush=True)


def species_states(nx, ny, tile, specs, seed, cell_box=None):
    return [pw.species_state(nx, ny, tile, s, seed, k, cell_box=cell_box) for k, s in enumerate(specs)]


def make_pair(nx, ny, dx, dy, dt, tile, specs, states, E=None, B=None, j_replicas=0, j_float=False, j_filter=0,
              esirkepov=False, sort_every=1, motion_sort=False, quadratic=False):
    """GPU Sim and OracleSim from the same FP32 initial state."""
    from paper_2501_14795_amd import Sim
    sim = Sim(nx, ny, dx, dy, dt, tile, [(s.qm, s.q, st) for s, st in zip(specs, states)], E=E, B=B,
              j_replicas=j_replicas, j_float=j_float, j_filter=j_filter, esirkepov=esirkepov, sort_every=sort_every,
              motion_sort=motion_sort, quadratic=quadratic)
    osp = [oracle.OracleSpecies(s.qm, s.q, st["ix"], st["iy"], st["x"], st["y"], st["ux"], st["uy"], st["uz"])
           for s, st in zip(specs, states)]
    ora = oracle.OracleSim(nx, ny, dx, dy, dt, osp,
                           None if E is None else E.astype(np.float64),
                           None if B is None else B.astype(np.float64), j_filter=j_filter, esirkepov=esirkepov,
                           quadratic=quadratic)
    return sim, ora


def oracle_from_gpu(sim, specs, dx, dy, dt):
    """OracleSim holding exactly the GPU's current FP32 state (replay)."""
    f = sim.field_arrays()
    osp = []
    for k, s in enumerate(specs):
        g = sim.state(k)
        osp.append(oracle.OracleSpecies(s.qm, s.q, g["ix"], g["iy"], g["x"], g["y"], g["ux"], g["uy"], g["uz"]))
    return oracle.OracleSim(sim.nx, sim.ny, dx, dy, dt, osp, f["E"].astype(np.float64),
                            f["B"].astype(np.float64))


def rel_err(a, b):
    den = np.abs(b).max()
    return float(np.abs(np.asarray(a, np.float64) - b).max() / (den if den > 0 else 1.0))


def particle_errors(g, o, nx, ny):
    """Element-by-element errors between GPU particles g (dict) and oracle
    species o, slot by slot.  Position error is measured on X = ix + x modulo
    the box (a face crossing decided differently in FP32 and FP64 changes the
    cell but not the position).  Returns (pos_err, u_rel_err)."""
    X = g["ix"] + g["x"].astype(np.float64)
    Y = g["iy"] + g["y"].astype(np.float64)
    Xo = o.ix + o.x
    Yo = o.iy + o.y
    dX = (X - Xo + nx / 2) % nx - nx / 2
    dY = (Y - Yo + ny / 2) % ny - ny / 2
    pos = max(np.abs(dX).max(initial=0.0), np.abs(dY).max(initial=0.0))
    umax = max(np.abs(o.ux).max(initial=0), np.abs(o.uy).max(initial=0), np.abs(o.uz).max(initial=0), 1e-30)
    du = max(np.abs(g["ux"] - o.ux).max(initial=0), np.abs(g["uy"] - o.uy).max(initial=0),
             np.abs(g["uz"] - o.uz).max(initial=0))
    return float(pos), float(du / umax)


def as_species(g):
    """A GPU state dict viewed like an OracleSpecies (FP64 offsets/momenta)."""
    class _S:
        pass
    s = _S()
    s.ix, s.iy = g["ix"], g["iy"]
    for k in ("x", "y", "ux", "uy", "uz"):
        setattr(s, k, g[k].astype(np.float64))
    return s


def matched_particle_errors(g, o, nx, ny):
    """Like particle_errors, but when the slot order differs (a tile crossing
    decided differently in FP32 and FP64 reorders a section) the particles are
    paired by nearest neighbour in (X, Y, u) space first."""
    pos, du = particle_errors(g, o, nx, ny)
    if pos < 1e-3:
        return pos, du, False
    from scipy.spatial import cKDTree
    Xg = np.c_[(g["ix"] + g["x"].astype(np.float64)) % nx, (g["iy"] + g["y"].astype(np.float64)) % ny]
    Xo = np.c_[(o.ix + o.x) % nx, (o.iy + o.y) % ny]
    # periodic in X, Y only: the tree needs non-negative coordinates and a
    # finite box, so u is shifted by a common offset into a box far larger
    # than its range
    Uo = np.c_[o.ux, o.uy, o.uz]
    Ug = np.c_[g["ux"], g["uy"], g["uz"]].astype(np.float64)
    lo = np.minimum(Uo.min(axis=0, initial=0.0), Ug.min(axis=0, initial=0.0))
    big = 1e9
    tree = cKDTree(np.c_[Xo, Uo - lo], boxsize=[nx, ny, big, big, big])
    _, idx = tree.query(np.c_[Xg, Ug - lo])
    assert len(np.unique(idx)) == len(idx), "nearest-neighbour pairing is not one-to-one"

    class _O:
        pass
    m = _O()
    for name in ("ix", "iy", "x", "y", "ux", "uy", "uz"):
        setattr(m, name, getattr(o, name)[idx])
    pos, du = particle_errors(g, m, nx, ny)
    return pos, du, True


def sort_replay(sim, specs, tile):
    """Run pic_sort and check it bit-exactly against the oracle's canonical
    sort of the GPU's own post-push cells."""
    pre = [sim.state(k) for k in range(len(specs))]
    sim.sort()
    assert sim.check() == 0
    for k in range(len(specs)):
        post = sim.state(k)
        off, src = oracle.sort_canonical(sim.nx, sim.ny, tile, pre[k]["ix"], pre[k]["iy"])
        assert np.array_equal(sim.tile_offsets(k), off), "tile_offset differs from the oracle"
        for name in PARTICLE_ARRAYS:
            assert np.array_equal(post[name], pre[k][name][src]), f"sorted {name} differs"
    return pre

"""FP64 CPU oracle for the 2D3V electromagnetic PIC step.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this package; the GPU library never does, and this
package imports nothing from it.  The arithmetic lives in ``pic_oracle.c``
(plain C, built with ``-ffp-contract=off``); this module only marshals numpy
arrays through ``ctypes``.

Every function follows a passage of the paper (Guidotti, "Accelerating
Particle-Mesh Algorithms with FPGAs and OmpSs@OpenCL"):

* ``interp``            -- linear interpolation on the staggered grid (Sec. 3.1)
* ``boris``             -- relativistic Boris push, Eqs. (6)-(10)
* ``deposit_move``      -- Villasenor-Buneman current, Eqs. (12)-(16), with the
                           1/2/3-piece split of Figs. 3.4-3.5
* ``deposit_esirkepov`` -- Esirkepov's charge-conserving current, the variant
                           deposit (density decomposition, linear shape)
* ``interp_quad`` / ``deposit_esirkepov_quad`` / ``rho(quadratic=True)`` -- the
                           quadratic B-spline shape for the gather, Esirkepov's
                           deposit and the node charge (an extension of the
                           linear weighting of Sec. 3.1; the paper has none)
* ``OracleSim.push_deposit`` -- the particle loop of Listing 3.1 + Eq. (11)
* ``yee_b`` / ``yee_e`` / ``OracleSim.field_advance`` -- Eqs. (19)-(20), the
                           three-step Yee update of Listing 3.1
* ``sort_canonical``    -- strict tile re-sort (Sec. 4.3, Fig. 4.5), with the
                           removed / appended particles of the moving window
* ``sort_motion_classes`` -- the alternative sort of Sec. 4.3 (after
                           Germaschewski et al.): regrouping by new tile in
                           one counting pass keyed on the motion class
* ``sort_stable_by_tile`` -- particles in any order grouped into the tile
                           sections of Sec. 4.1 (Fig. 4.3), keeping their order
                           within a tile (numpy's stable sort, Python)
* ``OracleSim.move_window`` -- the moving-window step of Listing 3.1
* ``binomial_filter``   -- the optional current smoothing of Listing 3.1
* ``rho`` / energies / divergences -- diagnostics (Eq. 17, Eq. 18, Eq. 12)
* ``solve_gauss``       -- valid initial fields (Sec. 3.2: Eqs. 17 and 18 hold
                           before the first step), by projection with an exact
                           periodic Poisson solve (numpy FFT, Python)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pic_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_SRC_OMP = os.path.join(_HERE, "pic_oracle_omp.c")
_SO_OMP = os.path.join(_HERE, "liboracle_omp.so")

_lib = None
_lib_omp = None

_d = ctypes.c_double
_i = ctypes.c_int
_i64 = ctypes.c_int64
_p = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile ``pic_oracle.c`` into ``liboracle.so`` with gcc (strict FP64)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
             "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def build_omp(force: bool = True) -> str:
    """Compile the OpenMP driver with the oracle into ``liboracle_omp.so``
    (the timed CPU baseline; the checker is ``liboracle.so``)."""
    if force or not os.path.exists(_SO_OMP):
        tmp = _SO_OMP + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
             "-o", tmp, _SRC, _SRC_OMP, "-lm"])
        os.replace(tmp, _SO_OMP)
    return _SO_OMP


def lib_omp():
    global _lib_omp
    if _lib_omp is None:
        if (not os.path.exists(_SO_OMP) or os.path.getmtime(_SO_OMP) < os.path.getmtime(_SRC_OMP)
                or os.path.getmtime(_SO_OMP) < os.path.getmtime(_SRC)):
            build_omp()
        L = ctypes.CDLL(_SO_OMP)
        L.ora_omp_threads.restype = _i
        L.ora_advance_omp.argtypes = [_i, _i, _d, _d, _d, _d, _d, _i64, _p] + [_p] * 7 + [_p] * 3
        L.ora_advance_omp.restype = _i
        L.ora_sort_canonical_omp.argtypes = [_i, _i, _i, _i64, _p, _p, _p, _p]
        L.ora_sort_canonical_omp.restype = _i
        L.ora_permute_omp.argtypes = [_i64, _p] + [_p] * 7
        L.ora_permute_omp.restype = _i
        _lib_omp = L
    return _lib_omp


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        L.ora_interp.argtypes = [_i, _i, _p, _p, _i, _i, _d, _d, _p]
        L.ora_boris.argtypes = [_d, _d, _p, _p]
        L.ora_deposit_move.argtypes = [_i, _i, _d, _d, _d, _d, _d, _i, _i, _d, _d, _d, _d, _p]
        L.ora_advance.argtypes = [_i, _i, _d, _d, _d, _d, _d, _i64] + [_p] * 10 + [_i]
        L.ora_deposit_esirkepov.argtypes = [_i, _i, _d, _d, _d, _d, _d, _i, _i, _d, _d, _d, _d, _p]
        L.ora_deposit_esirkepov_quad.argtypes = [_i, _i, _d, _d, _d, _d, _d, _i, _i, _d, _d, _d, _d, _p]
        L.ora_interp_quad.argtypes = [_i, _i, _p, _p, _i, _i, _d, _d, _p]
        L.ora_deposit_rho_quad.argtypes = [_i, _i, _d, _i64, _p, _p, _p, _p, _p]
        L.ora_advance.restype = _i
        L.ora_yee_b.argtypes = [_i, _i, _d, _d, _d, _p, _p]
        L.ora_yee_e.argtypes = [_i, _i, _d, _d, _d, _p, _p, _p]
        L.ora_field_advance.argtypes = [_i, _i, _d, _d, _d, _p, _p, _p]
        L.ora_sort_canonical.argtypes = [_i, _i, _i, _i64, _p, _p, _p, _p, _p, _p]
        L.ora_sort_canonical.restype = _i
        L.ora_sort_motion_classes.argtypes = [_i, _i, _i, _i64, _p, _p, _p, _p, _p]
        L.ora_sort_motion_classes.restype = _i
        L.ora_deposit_rho.argtypes = [_i, _i, _d, _i64, _p, _p, _p, _p, _p]
        L.ora_field_energy.argtypes = [_i, _i, _d, _d, _p]
        L.ora_field_energy.restype = _d
        L.ora_kinetic_energy.argtypes = [_d, _d, _d, _d, _i64, _p, _p, _p]
        L.ora_kinetic_energy.restype = _d
        L.ora_div_e.argtypes = [_i, _i, _d, _d, _p, _p]
        L.ora_div_b.argtypes = [_i, _i, _d, _d, _p, _p]
        L.ora_binomial_filter.argtypes = [_i, _i, _i, _i64, _p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


# --------------------------------------------------------------------------
# single-particle / single-operator entry points (used by the pins)
# --------------------------------------------------------------------------

def interp(nx, ny, E, B, ix, iy, x, y) -> np.ndarray:
    """{Ex,Ey,Ez,Bx,By,Bz} at one particle; E, B are (3, ny, nx) arrays."""
    E = _f64(E)
    B = _f64(B)
    out = np.zeros(6)
    lib().ora_interp(nx, ny, _ptr(E), _ptr(B), int(ix), int(iy), float(x), float(y), _ptr(out))
    return out


def interp_quad(nx, ny, E, B, ix, iy, x, y) -> np.ndarray:
    """{Ex,Ey,Ez,Bx,By,Bz} at one particle with the quadratic shape."""
    E = _f64(E)
    B = _f64(B)
    out = np.zeros(6)
    lib().ora_interp_quad(nx, ny, _ptr(E), _ptr(B), int(ix), int(iy), float(x), float(y), _ptr(out))
    return out


def boris(qm, dt, EB, u) -> np.ndarray:
    """One Boris update of u(t-dt/2) -> u(t+dt/2) in the fields EB = (E, B)."""
    EB = _f64(EB)
    u = _f64(u).copy()
    lib().ora_boris(float(qm), float(dt), _ptr(EB), _ptr(u))
    return u


def deposit_move(nx, ny, dx, dy, dt, q, vz, ix, iy, x, y, ddx, ddy, J=None) -> np.ndarray:
    """Current (3, ny, nx) of one straight move by (ddx, ddy) cells."""
    if J is None:
        J = np.zeros((3, ny, nx))
    lib().ora_deposit_move(nx, ny, dx, dy, dt, q, vz, int(ix), int(iy), float(x), float(y),
                           float(ddx), float(ddy), _ptr(J))
    return J


def deposit_esirkepov(nx, ny, dx, dy, dt, q, vz, ix, iy, x, y, ddx, ddy, J=None) -> np.ndarray:
    """Esirkepov current (3, ny, nx) of one straight move by (ddx, ddy) cells."""
    if J is None:
        J = np.zeros((3, ny, nx))
    lib().ora_deposit_esirkepov(nx, ny, dx, dy, dt, q, vz, int(ix), int(iy), float(x), float(y),
                                float(ddx), float(ddy), _ptr(J))
    return J


def deposit_esirkepov_quad(nx, ny, dx, dy, dt, q, vz, ix, iy, x, y, ddx, ddy, J=None) -> np.ndarray:
    """Esirkepov current (3, ny, nx) of one straight move with the quadratic shape."""
    if J is None:
        J = np.zeros((3, ny, nx))
    lib().ora_deposit_esirkepov_quad(nx, ny, dx, dy, dt, q, vz, int(ix), int(iy), float(x), float(y),
                                     float(ddx), float(ddy), _ptr(J))
    return J


def yee_b(nx, ny, dx, dy, h, E, B):
    lib().ora_yee_b(nx, ny, dx, dy, h, _ptr(E), _ptr(B))


def yee_e(nx, ny, dx, dy, h, B, J, E):
    lib().ora_yee_e(nx, ny, dx, dy, h, _ptr(B), _ptr(J), _ptr(E))


def sort_canonical(nx, ny, T, ix, iy, removed=None):
    """Canonical strict tile sort.  Returns (off[ntiles+1], src[n']) as int64;
    `removed` (bool array or None) marks particles that belong to no tile."""
    ix = _i32(ix)
    iy = _i32(iy)
    n = ix.size
    ntiles = (nx // T) * (ny // T)
    off = np.zeros(ntiles + 1, dtype=np.int64)
    src = np.zeros(max(n, 1), dtype=np.int64)
    n_out = np.zeros(1, dtype=np.int64)
    rm = None if removed is None else np.ascontiguousarray(removed, dtype=np.uint8)
    rc = lib().ora_sort_canonical(nx, ny, T, n, _ptr(ix), _ptr(iy), None if rm is None else _ptr(rm), _ptr(off),
                                  _ptr(src), _ptr(n_out))
    if rc != 0:
        raise ValueError("cell index out of range")
    return off, src[:int(n_out[0])]


def sort_motion_classes(nx, ny, T, ix, iy, off_old):
    """The motion-class sort: particles in their tile sections (off_old, the
    tile_offset before the sort) with cells (ix, iy) after the push, ordered
    by (new tile, motion class, old slot); the class of a particle moving from
    tile s to tile t is (dty + 1) * 3 + (dtx + 1), (dtx, dty) the step on the
    periodic tile grid (+1 when an axis has two tiles).  Returns (new
    tile_offset, src) with src[j] the old slot of the particle at slot j."""
    ix, iy = _i32(ix), _i32(iy)
    n = ix.size
    ntiles = (nx // T) * (ny // T)
    oo = np.ascontiguousarray(off_old, dtype=np.int64)
    assert oo.size == ntiles + 1 and oo[-1] == n
    off = np.zeros(ntiles + 1, dtype=np.int64)
    src = np.zeros(max(n, 1), dtype=np.int64)
    rc = lib().ora_sort_motion_classes(nx, ny, T, n, _ptr(ix), _ptr(iy), _ptr(oo), _ptr(off), _ptr(src))
    if rc != 0:
        raise ValueError("a cell is outside the grid or more than one tile from its section")
    return off, src[:n]


def sort_stable_by_tile(nx, ny, T, ix, iy):
    """Particles in any order grouped by tile (Sec. 4.1: the particles of a
    tile occupy one section, sections in tile order, Fig. 4.3), the given
    order kept inside each tile.  Tiles are numbered row-major.  Returns
    (off[ntiles+1], src) with the grouped arrays = arrays[src]."""
    ix = _i32(ix)
    iy = _i32(iy)
    if ix.size and (ix.min() < 0 or ix.max() >= nx or iy.min() < 0 or iy.max() >= ny):
        raise ValueError("cell index out of range")
    ntx = nx // T
    tile = (iy // T).astype(np.int64) * ntx + ix // T
    src = np.argsort(tile, kind="stable")
    off = np.r_[0, np.cumsum(np.bincount(tile, minlength=ntx * (ny // T)))].astype(np.int64)
    return off, src


def rho(nx, ny, q, ix, iy, x, y, out=None, quadratic=False) -> np.ndarray:
    """Node charge density (ny, nx) of one species (accumulates into out),
    with the linear or the quadratic shape."""
    if out is None:
        out = np.zeros((ny, nx))
    ix = _i32(ix)
    iy = _i32(iy)
    x = _f64(x)
    y = _f64(y)
    f = lib().ora_deposit_rho_quad if quadratic else lib().ora_deposit_rho
    f(nx, ny, q, ix.size, _ptr(ix), _ptr(iy), _ptr(x), _ptr(y), _ptr(out))
    return out


def field_energy(nx, ny, dx, dy, F) -> float:
    F = _f64(F)
    return lib().ora_field_energy(nx, ny, dx, dy, _ptr(F))


def kinetic_energy(dx, dy, qm, q, ux, uy, uz) -> float:
    ux, uy, uz = _f64(ux), _f64(uy), _f64(uz)
    return lib().ora_kinetic_energy(dx, dy, qm, q, ux.size, _ptr(ux), _ptr(uy), _ptr(uz))


def div_e(nx, ny, dx, dy, F) -> np.ndarray:
    F = _f64(F)
    out = np.zeros((ny, nx))
    lib().ora_div_e(nx, ny, dx, dy, _ptr(F), _ptr(out))
    return out


def div_b(nx, ny, dx, dy, B) -> np.ndarray:
    B = _f64(B)
    out = np.zeros((ny, nx))
    lib().ora_div_b(nx, ny, dx, dy, _ptr(B), _ptr(out))
    return out


def binomial_filter(nx, ny, passes, F):
    """In place: `passes` binomial (1/4, 1/2, 1/4) passes, x then y, on each
    (ny, nx) plane of the FP64 array F (shape (ny, nx) or (k, ny, nx))."""
    if F.dtype != np.float64 or not F.flags.c_contiguous or F.shape[-2:] != (ny, nx):
        raise ValueError("F must be a C-contiguous float64 array of (..., ny, nx) planes")
    lib().ora_binomial_filter(nx, ny, int(passes), F.size // (nx * ny), _ptr(F))
    return F


def poisson_periodic(nx, ny, dx, dy, r) -> np.ndarray:
    """The zero-mean psi (ny, nx) whose five-point Laplacian
    (psi[i+1] - 2 psi[i] + psi[i-1]) / dx^2 + (same along y) / dy^2 equals r
    on the periodic grid (r must have zero mean).  Exact: the discrete
    Fourier modes diagonalise the operator, with eigenvalues
    -(2 - 2 cos(2 pi m / nx)) / dx^2 - (2 - 2 cos(2 pi l / ny)) / dy^2."""
    r = np.asarray(r, np.float64)
    m = np.arange(nx)
    l = np.arange(ny)
    lam = (-(2.0 - 2.0 * np.cos(2.0 * np.pi * m / nx)) / (dx * dx))[None, :] + \
          (-(2.0 - 2.0 * np.cos(2.0 * np.pi * l / ny)) / (dy * dy))[:, None]
    lam[0, 0] = 1.0
    h = np.fft.fft2(r) / lam
    h[0, 0] = 0.0
    return np.real(np.fft.ifft2(h))


def solve_gauss(nx, ny, dx, dy, E, B, rho_nodes):
    """Valid initial fields (Sec. 3.2: the fields start satisfying Eq. 17,
    div E = rho, and Eq. 18, div B = 0), in place on FP64 E, B (3, ny, nx).
    With the ions as a uniform background the charge is rho - mean(rho).
    E <- E - grad psi with Lap psi = div E - (rho - mean(rho)) (psi at the
    nodes; Ex at (i+1/2, j) takes (psi[i+1] - psi[i]) / dx, Ey likewise);
    B <- B - grad chi with Lap chi = div B (chi at the cell centres; Bx at
    (i, j+1/2) takes (chi[i] - chi[i-1]) / dx, By likewise).  A gradient has
    no discrete curl on the Yee grid, so the curls of E and B -- what drives
    Eqs. 19 and 20 -- are unchanged; with E = 0 on entry this is the
    electrostatic field of the charge."""
    rho_nodes = np.asarray(rho_nodes, np.float64)
    r = div_e(nx, ny, dx, dy, E) - (rho_nodes - rho_nodes.mean())
    psi = poisson_periodic(nx, ny, dx, dy, r - r.mean())
    E[0] -= (np.roll(psi, -1, axis=1) - psi) / dx
    E[1] -= (np.roll(psi, -1, axis=0) - psi) / dy
    s = div_b(nx, ny, dx, dy, B)
    chi = poisson_periodic(nx, ny, dx, dy, s - s.mean())
    B[0] -= (chi - np.roll(chi, 1, axis=1)) / dx
    B[1] -= (chi - np.roll(chi, 1, axis=0)) / dy
    return E, B


# --------------------------------------------------------------------------
# whole-simulation driver
# --------------------------------------------------------------------------

class OracleSpecies:
    """Particles of one species, FP64 offsets and momenta, int32 cells."""

    def __init__(self, qm, q, ix, iy, x, y, ux, uy, uz):
        self.qm = float(qm)
        self.q = float(q)
        self.ix = _i32(ix).copy()
        self.iy = _i32(iy).copy()
        self.x = _f64(x).copy()
        self.y = _f64(y).copy()
        self.ux = _f64(ux).copy()
        self.uy = _f64(uy).copy()
        self.uz = _f64(uz).copy()

    @property
    def n(self):
        return self.ix.size

    def permute(self, src):
        for name in ("ix", "iy", "x", "y", "ux", "uy", "uz"):
            setattr(self, name, np.ascontiguousarray(getattr(self, name)[src]))


class OracleSim:
    """Serial FP64 PIC on a periodic nx x ny grid (Listing 3.1 order)."""

    def __init__(self, nx, ny, dx, dy, dt, species, E=None, B=None, j_filter=0, esirkepov=False,
                 quadratic=False):
        self.nx, self.ny = int(nx), int(ny)
        self.j_filter = int(j_filter)
        self.esirkepov = bool(esirkepov)
        self.quadratic = bool(quadratic)   # quadratic shape: gather and Esirkepov deposit
        self.dx, self.dy, self.dt = float(dx), float(dy), float(dt)
        self.species = list(species)
        shape = (3, self.ny, self.nx)
        self.E = np.zeros(shape) if E is None else _f64(E).reshape(shape).copy()
        self.B = np.zeros(shape) if B is None else _f64(B).reshape(shape).copy()
        self.J = np.zeros(shape)

    def push_deposit(self):
        """Zero J, then interpolate / push / move / deposit every particle."""
        self.J[...] = 0.0
        for s in self.species:
            rc = lib().ora_advance(self.nx, self.ny, self.dx, self.dy, self.dt, s.qm, s.q, s.n,
                                   _ptr(s.ix), _ptr(s.iy), _ptr(s.x), _ptr(s.y),
                                   _ptr(s.ux), _ptr(s.uy), _ptr(s.uz),
                                   _ptr(self.E), _ptr(self.B), _ptr(self.J),
                                   2 if self.quadratic else int(self.esirkepov))
            if rc != 0:
                raise FloatingPointError("a particle moved one cell or more (Courant condition)")
        if self.j_filter:
            binomial_filter(self.nx, self.ny, self.j_filter, self.J)

    def field_advance(self):
        lib().ora_field_advance(self.nx, self.ny, self.dx, self.dy, self.dt,
                                _ptr(self.E), _ptr(self.B), _ptr(self.J))

    def sort(self, T):
        """Canonical tile sort of every species; returns the new offsets."""
        offs = []
        for s in self.species:
            off, src = sort_canonical(self.nx, self.ny, T, s.ix, s.iy)
            s.permute(src)
            offs.append(off)
        return offs

    def step(self, T=None):
        self.push_deposit()
        if T is not None:
            self.sort(T)
        self.field_advance()

    def move_window(self, inject, T):
        """The moving-window step at the end of Listing 3.1: E and B move one
        cell towards -x (the new last column is zero), every particle moves one
        cell towards -x (ix - 1, offsets kept), the particles that were in
        column 0 leave, and the new particles `inject` (one dict of ix, iy, x,
        y, ux, uy, uz arrays per species, all in column nx - 1) come in.  The
        particles are then re-sorted canonically by tile, the new ones counted
        as appended after the existing ones, the leaving ones as removed."""
        for F in (self.E, self.B):
            F[:, :, :-1] = F[:, :, 1:].copy()
            F[:, :, -1] = 0.0
        for s, inj in zip(self.species, inject):
            ix = s.ix - 1
            removed = ix < 0
            ix = np.where(removed, 0, ix)
            cat = {"ix": np.r_[ix, _i32(inj["ix"])], "iy": np.r_[s.iy, _i32(inj["iy"])]}
            for name in ("x", "y", "ux", "uy", "uz"):
                cat[name] = np.r_[getattr(s, name), _f64(inj[name])]
            rm = np.r_[removed, np.zeros(len(inj["ix"]), bool)]
            _, src = sort_canonical(self.nx, self.ny, T, cat["ix"], cat["iy"], removed=rm)
            for name, v in cat.items():
                setattr(s, name, np.ascontiguousarray(v[src], dtype=np.int32 if name in ("ix", "iy") else np.float64))

    def solve_gauss(self):
        """Make E and B valid initial fields for the current particles
        (``solve_gauss``)."""
        solve_gauss(self.nx, self.ny, self.dx, self.dy, self.E, self.B, self.rho())

    def rho(self, filtered=False):
        """Node charge density; with filtered=True smoothed by the current filter
        (the density whose continuity the filtered current satisfies)."""
        r = np.zeros((self.ny, self.nx))
        for s in self.species:
            rho(self.nx, self.ny, s.q, s.ix, s.iy, s.x, s.y, out=r, quadratic=self.quadratic)
        if filtered and self.j_filter:
            binomial_filter(self.nx, self.ny, self.j_filter, r)
        return r

    def energies(self):
        ue = field_energy(self.nx, self.ny, self.dx, self.dy, self.E)
        ub = field_energy(self.nx, self.ny, self.dx, self.dy, self.B)
        uk = [kinetic_energy(self.dx, self.dy, s.qm, s.q, s.ux, s.uy, s.uz) for s in self.species]
        return ue, ub, uk


# --------------------------------------------------------------------------
# the OpenMP driver (timed CPU baseline, not a checker)
# --------------------------------------------------------------------------

def omp_threads() -> int:
    """Threads the OpenMP driver uses (OMP_NUM_THREADS, else every core)."""
    return int(lib_omp().ora_omp_threads())


def sort_canonical_omp(nx, ny, T, ix, iy):
    """sort_canonical (no removed particles) computed by the OpenMP driver."""
    ix, iy = _i32(ix), _i32(iy)
    n = ix.size
    ntiles = (nx // T) * (ny // T)
    off = np.zeros(ntiles + 1, dtype=np.int64)
    src = np.zeros(max(n, 1), dtype=np.int64)
    if lib_omp().ora_sort_canonical_omp(nx, ny, T, n, _ptr(ix), _ptr(iy), _ptr(off), _ptr(src)) != 0:
        raise ValueError("cell index out of range")
    return off, src[:n]


class OracleOmpSim(OracleSim):
    """OracleSim whose particle half runs tile-parallel with OpenMP (Sec.
    4.2.1: an OpenMP loop over the tiles, a private current per thread) and
    whose strict sort is computed with the work split over threads.  The
    particles must be grouped by tiles of T x T cells (they are after every
    sort).  Same results as OracleSim to FP64 round-off (the sort bit for
    bit); Villasenor-Buneman deposit, no filter."""

    def __init__(self, nx, ny, dx, dy, dt, species, T, E=None, B=None):
        super().__init__(nx, ny, dx, dy, dt, species, E, B)
        self.T = int(T)
        self.offs = [self._offsets(s) for s in self.species]

    def _offsets(self, s):
        ntx = self.nx // self.T
        tile = (s.iy // self.T).astype(np.int64) * ntx + s.ix // self.T
        if tile.size and (np.diff(tile) < 0).any():
            raise ValueError("particles are not grouped by tile")
        return np.searchsorted(tile, np.arange((self.ny // self.T) * ntx + 1)).astype(np.int64)

    def push_deposit(self):
        self.J[...] = 0.0
        ntiles = (self.nx // self.T) * (self.ny // self.T)
        for s, off in zip(self.species, self.offs):
            rc = lib_omp().ora_advance_omp(self.nx, self.ny, self.dx, self.dy, self.dt, s.qm, s.q, ntiles,
                                           _ptr(off), _ptr(s.ix), _ptr(s.iy), _ptr(s.x), _ptr(s.y),
                                           _ptr(s.ux), _ptr(s.uy), _ptr(s.uz),
                                           _ptr(self.E), _ptr(self.B), _ptr(self.J))
            if rc != 0:
                raise FloatingPointError("a particle moved one cell or more (Courant condition)")

    def sort(self, T=None):
        offs = []
        for k, s in enumerate(self.species):
            off, src = sort_canonical_omp(self.nx, self.ny, self.T, s.ix, s.iy)
            src = np.ascontiguousarray(src, dtype=np.int64)
            if lib_omp().ora_permute_omp(s.n, _ptr(src), _ptr(s.ix), _ptr(s.iy), _ptr(s.x), _ptr(s.y),
                                         _ptr(s.ux), _ptr(s.uy), _ptr(s.uz)) != 0:
                raise MemoryError("ora_permute_omp")
            self.offs[k] = off
            offs.append(off)
        return offs

"""Pins of the oracle's quadratic particle shape (the higher-order variant of
the linear weighting of Sec. 3.1: the gather, Esirkepov's deposit and the node
charge with the second-order B-spline).

The independent definition here is the node charge of a triangular cloud of
half-width one cell (the linear shape as a charge distribution) collected on
the node dual cells [i-1/2, i+1/2], by integrating the triangle over each dual
cell (numpy, closed-form antiderivative).  It must equal the oracle's
quadratic shape weight; on top of it the pins use closed forms (moments of the
shape, totals of the current), charge continuity (Eq. 12) with that charge,
exact reproduction of bilinear fields by the gather, and the mirror and
transposition symmetries of the deposit.  A wrong stagger offset, a wrong
weight branch, a dropped term of W^x / W^y / W^z or a stencil that misses a
node fails at least one of them."""
import math

import numpy as np
import pytest

import pic_workloads as pw

STAGGER = [(0.5, 0.0), (0.0, 0.5), (0.0, 0.0),   # Ex Ey Ez
           (0.0, 0.5), (0.5, 0.0), (0.5, 0.5)]   # Bx By Bz


@pytest.fixture(scope="module")
def ora():
    import oracle
    oracle.build(force=False)
    return oracle


def tent_cdf(u):
    """Integral of the unit triangle max(0, 1 - |s|) from -inf to u."""
    u = np.asarray(u, np.float64)
    return np.where(u < -1, 0.0, np.where(u < 0, 0.5 * (1 + u) ** 2,
                                          np.where(u < 1, 1 - 0.5 * (1 - u) ** 2, 1.0)))


def tsc_weights(X, n):
    """Charge of a triangular cloud centred at X on the dual cells of nodes
    0..n-1 of a periodic axis (images at X +- n included)."""
    i = np.arange(n)
    w = np.zeros(n)
    for shift in (-n, 0, n):
        w += tent_cdf(i + 0.5 - (X + shift)) - tent_cdf(i - 0.5 - (X + shift))
    return w


def tsc_charge(nx, ny, q, X, Y):
    """Node charge (ny, nx) of triangular clouds at (X, Y)."""
    rho = np.zeros((ny, nx))
    for Xc, Yc in zip(np.atleast_1d(X), np.atleast_1d(Y)):
        rho += q * np.outer(tsc_weights(Yc, ny), tsc_weights(Xc, nx))
    return rho


def div_edge(J, dx, dy):
    return (J[0] - np.roll(J[0], 1, axis=1)) / dx + (J[1] - np.roll(J[1], 1, axis=0)) / dy


def new_position(nx, ny, ix, iy, x, y, ddx, ddy):
    return (ix + x + ddx) % nx, (iy + y + ddy) % ny


def _cases(rng, n_random=40):
    cases = [(3, 3, 0.5, 0.5, 0.0, 0.0), (3, 3, 0.49, 0.51, 0.02, -0.03), (3, 3, 0.9, 0.1, 0.95, -0.95),
             (3, 3, 0.05, 0.95, -0.9, 0.9), (3, 3, 0.5, 0.5, 0.5, 0.0), (3, 3, 0.0, 0.0, -0.999, -0.999),
             (0, 0, 0.1, 0.2, -0.6, -0.7), (7, 7, 0.95, 0.9, 0.6, 0.7), (4, 2, 0.7, 0.3, 0.8, -0.5)]
    for _ in range(n_random):
        ix, iy = rng.integers(0, 8, 2)
        x, y = rng.uniform(0, 1, 2)
        ddx, ddy = rng.uniform(-0.99, 0.99, 2)
        cases.append((int(ix), int(iy), x, y, ddx, ddy))
    return cases


def test_quadratic_charge_is_the_triangular_cloud(ora):
    """The oracle's quadratic node charge equals the triangular cloud's charge
    on the dual cells (also across the periodic seam), and its moments are
    the B-spline's: total q, centre X, variance 1/4 of a cell squared."""
    nx, ny, q = 8, 6, -0.37
    rng = np.random.default_rng(31)
    for _ in range(200):
        ix, iy = int(rng.integers(0, nx)), int(rng.integers(0, ny))
        x, y = rng.uniform(0, 1, 2)
        r = ora.rho(nx, ny, q, np.array([ix]), np.array([iy]), np.array([x]), np.array([y]), quadratic=True)
        np.testing.assert_allclose(r, tsc_charge(nx, ny, q, ix + x, iy + y), atol=1e-15)
    # moments away from the seam
    for X in rng.uniform(2, 5, 50):
        w = ora.rho(8, 1, 1.0, np.array([int(X)]), np.array([0]), np.array([X - int(X)]), np.array([0.0]),
                    quadratic=True)[0] / tsc_weights(0.0, 1)[0]
        i = np.arange(8)
        assert abs(w.sum() - 1.0) < 1e-14
        assert abs((i * w).sum() - X) < 1e-13
        assert abs((i * i * w).sum() - (X * X + 0.25)) < 1e-12
    # the linear shape is a different charge
    r1 = ora.rho(nx, ny, q, np.array([3]), np.array([2]), np.array([0.3]), np.array([0.6]))
    r2 = ora.rho(nx, ny, q, np.array([3]), np.array([2]), np.array([0.3]), np.array([0.6]), quadratic=True)
    assert np.abs(r1 - r2).max() > 0.02 * abs(q)


def _polynomial_fields(nx, ny, coef):
    """E, B whose component c samples f_c(X, Y) = a + bX + cY + dXY at its own
    staggered points (X = i + sx, Y = j + sy)."""
    F = np.zeros((6, ny, nx))
    j, i = np.mgrid[0:ny, 0:nx].astype(np.float64)
    for c, (sx, sy) in enumerate(STAGGER):
        a, b, cc, d = coef[c]
        X, Y = i + sx, j + sy
        F[c] = a + b * X + cc * Y + d * X * Y
    return F[:3], F[3:]


def test_quadratic_gather_reproduces_bilinear_fields(ora):
    """The quadratic B-spline reproduces polynomials of degree one per axis:
    every component of a field a + bX + cY + dXY (sampled at its staggered
    points) is interpolated exactly at any particle position inside the
    grid; a stagger offset off by half a cell would be off by b/2."""
    nx = ny = 12
    rng = np.random.default_rng(32)
    coef = rng.uniform(-1, 1, (6, 4))
    E, B = _polynomial_fields(nx, ny, coef)
    for _ in range(200):
        ix, iy = rng.integers(2, 9, 2)
        x, y = rng.uniform(0, 1, 2)
        X, Y = ix + x, iy + y
        got = ora.interp_quad(nx, ny, E, B, ix, iy, x, y)
        want = [a + b * X + c * Y + d * X * Y for a, b, c, d in coef]
        np.testing.assert_allclose(got, want, atol=1e-12)


def test_quadratic_gather_second_moment(ora):
    """Sampled X^2 (and Y^2) comes back as X^2 + 1/4: the B-spline's variance,
    which distinguishes it from quadratic Lagrange interpolation (X^2
    exactly) and from the linear weighting (X^2 + f(1 - f))."""
    nx = ny = 12
    j, i = np.mgrid[0:ny, 0:nx].astype(np.float64)
    rng = np.random.default_rng(33)
    for c, (sx, sy) in enumerate(STAGGER):
        F = np.zeros((6, ny, nx))
        F[c] = (i + sx) ** 2 + 2.0 * (j + sy) ** 2
        for _ in range(40):
            ix, iy = rng.integers(2, 9, 2)
            x, y = rng.uniform(0, 1, 2)
            X, Y = ix + x, iy + y
            got = ora.interp_quad(nx, ny, F[:3], F[3:], ix, iy, x, y)[c]
            assert abs(got - (X * X + 0.25 + 2.0 * (Y * Y + 0.25))) < 1e-11, (c, X, Y)


def test_quadratic_deposit_continuity_and_totals(ora):
    """Esirkepov's decomposition with the quadratic shape conserves the
    triangular cloud's node charge exactly, Eq. (12), for every motion, and
    moves the whole charge: sum Jx dt/dx = q ddx, sum Jy dt/dy = q ddy,
    sum Jz = q vz."""
    nx, ny, dx, dy, dt, q, vz = 8, 8, 0.1, 0.1, 0.07, -0.37, 0.3
    rng = np.random.default_rng(34)
    for ix, iy, x, y, ddx, ddy in _cases(rng):
        J = ora.deposit_esirkepov_quad(nx, ny, dx, dy, dt, q, vz, ix, iy, x, y, ddx, ddy)
        X1, Y1 = new_position(nx, ny, ix, iy, x, y, ddx, ddy)
        res = tsc_charge(nx, ny, q, X1, Y1) - tsc_charge(nx, ny, q, ix + x, iy + y) + dt * div_edge(J, dx, dy)
        assert np.abs(res).max() < 1e-13, (ix, iy, x, y, ddx, ddy)
        assert abs(J[0].sum() * dt / dx - q * ddx) < 1e-14
        assert abs(J[1].sum() * dt / dy - q * ddy) < 1e-14
        assert abs(J[2].sum() - q * vz) < 1e-14


def test_quadratic_deposit_special_cases(ora):
    """(1) No motion: no in-plane current, and Jz = q vz times the charge
    weights.  (2) Motion along x only: Jx on row l is the triangular cloud's
    charge crossing each x face times its weight on row l; no Jy.
    (3) Mirroring x (X -> -X, ddx -> -ddx) mirrors Jy and Jz and turns Jx
    around.  (4) Exchanging x and y exchanges Jx and Jy and transposes.
    (5) Not the linear-shape current."""
    nx, ny, dx, dy, dt, q, vz = 8, 8, 0.1, 0.1, 0.07, 0.5, -0.4
    rng = np.random.default_rng(35)
    for _ in range(50):
        x, y = rng.uniform(0, 1, 2)
        J = ora.deposit_esirkepov_quad(nx, ny, dx, dy, dt, q, vz, 3, 4, x, y, 0.0, 0.0)
        assert np.abs(J[:2]).max() == 0.0
        np.testing.assert_allclose(J[2], vz * tsc_charge(nx, ny, q, 3 + x, 4 + y), atol=1e-15)
    for _ in range(50):
        x, y = rng.uniform(0, 1, 2)
        ddx = rng.uniform(-0.99, 0.99)
        J = ora.deposit_esirkepov_quad(nx, ny, dx, dy, dt, q, vz, 3, 4, x, y, ddx, 0.0)
        w0, w1 = tsc_weights(3 + x, nx), tsc_weights(3 + x + ddx, nx)
        # charge to the right of face k + 1/2 after minus before (no wrap here)
        flux = np.array([(w1[k + 1:] - w0[k + 1:]).sum() for k in range(nx)])
        wy = tsc_weights(4 + y, ny)
        np.testing.assert_allclose(J[0] * dt / dx, q * np.outer(wy, flux), atol=1e-15)
        assert np.abs(J[1]).max() == 0.0
    for _ in range(50):
        ix, iy = 3, 4
        x, y = rng.uniform(0.01, 0.99, 2)
        ddx, ddy = rng.uniform(-0.99, 0.99, 2)
        A = ora.deposit_esirkepov_quad(nx, ny, dx, dy, dt, q, vz, ix, iy, x, y, ddx, ddy)
        # mirror: X' = -X = (-ix - 1) + (1 - x), node i -> -i, face i+1/2 -> -i-1/2
        M = ora.deposit_esirkepov_quad(nx, ny, dx, dy, dt, q, vz, (-ix - 1) % nx, iy, 1.0 - x, y, -ddx, ddy)
        idx = (-np.arange(nx)) % nx
        np.testing.assert_allclose(M[0][:, (-np.arange(nx) - 1) % nx], -A[0], atol=1e-14)
        np.testing.assert_allclose(M[1][:, idx], A[1], atol=1e-14)
        np.testing.assert_allclose(M[2][:, idx], A[2], atol=1e-14)
        Bt = ora.deposit_esirkepov_quad(ny, nx, dy, dx, dt, q, vz, iy, ix, y, x, ddy, ddx)
        np.testing.assert_allclose(A[0], Bt[1].T, atol=1e-14)
        np.testing.assert_allclose(A[1], Bt[0].T, atol=1e-14)
        np.testing.assert_allclose(A[2], Bt[2].T, atol=1e-14)
    Jq = ora.deposit_esirkepov_quad(nx, ny, dx, dy, dt, q, vz, 3, 4, 0.3, 0.6, 0.2, 0.1)
    Jl = ora.deposit_esirkepov(nx, ny, dx, dy, dt, q, vz, 3, 4, 0.3, 0.6, 0.2, 0.1)
    assert np.abs(Jq - Jl).max() > 1e-3 * abs(q) * dx / dt


def test_quadratic_whole_step_gauss(ora):
    """Full steps with the quadratic shape keep Gauss's law (div E minus the
    triangular cloud's charge) at its initial residual."""
    nx = ny = 16
    spec = pw.SpeciesSpec(-1.0, (2, 2), (0.2, 0.2, 0.2), (0.1, 0.0, 0.0))
    st = pw.species_state(nx, ny, 4, spec, 36)
    sp = ora.OracleSpecies(spec.qm, spec.q, st["ix"], st["iy"], st["x"], st["y"], st["ux"], st["uy"], st["uz"])
    E, B = pw.random_fields(nx, ny, 0.05, 36)
    sim = ora.OracleSim(nx, ny, 0.1, 0.1, 0.07, [sp], E, B, quadratic=True)
    s = sim.species[0]

    def gauss():
        X, Y = s.ix + s.x, s.iy + s.y
        return div_edge(sim.E, sim.dx, sim.dy) - tsc_charge(nx, ny, s.q, X, Y)

    g0 = gauss()
    np.testing.assert_allclose(sim.rho(), tsc_charge(nx, ny, s.q, s.ix + s.x, s.iy + s.y), atol=1e-13)
    for _ in range(8):
        sim.push_deposit()
        sim.field_advance()
    assert np.abs(gauss() - g0).max() < 1e-11
    assert math.isfinite(sim.energies()[0])

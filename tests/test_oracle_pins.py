"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expected value is a closed
form, an invariant, a textbook special case or a brute-force computation done
independently in numpy (area flux of the unit-square cloud, node charge of the
cloud, discrete divergence).  A dropped term, a wrong sign or a transposed
operand in the oracle fails at least one of these.
"""
import math

import numpy as np
import pytest

# Staggered sample points of the six components (standard 2D Yee layout; the
# paper's Fig. 3.1 is lost): (sx, sy) such that F[i, j] lives at (i+sx, j+sy).
STAGGER = [(0.5, 0.0), (0.0, 0.5), (0.0, 0.0),   # Ex Ey Ez
           (0.0, 0.5), (0.5, 0.0), (0.5, 0.5)]   # Bx By Bz


# ---------------------------------------------------------------- helpers
def node_charge(nx, ny, q, X, Y):
    """Charge of unit-square clouds centred at (X, Y) (cell units) on the node
    dual cells [i-1/2, i+1/2] x [j-1/2, j+1/2]: overlap areas, by definition."""
    rho = np.zeros((ny, nx))
    for Xc, Yc in zip(np.atleast_1d(X), np.atleast_1d(Y)):
        i0, j0 = int(math.floor(Xc)), int(math.floor(Yc))
        for i in range(i0 - 1, i0 + 3):
            ox = max(0.0, min(Xc + 0.5, i + 0.5) - max(Xc - 0.5, i - 0.5))
            for j in range(j0 - 1, j0 + 3):
                oy = max(0.0, min(Yc + 0.5, j + 0.5) - max(Yc - 0.5, j - 0.5))
                rho[j % ny, i % nx] += q * ox * oy
    return rho


def div_edge(J, dx, dy):
    """Divergence at the nodes of a field living on (i+1/2, j) / (i, j+1/2)."""
    return (J[0] - np.roll(J[0], 1, axis=1)) / dx + (J[1] - np.roll(J[1], 1, axis=0)) / dy


def brute_current(nx, ny, dx, dy, dt, q, vz, X0, Y0, ddx, ddy, nsub=200000):
    """Current of a unit-square cloud moving straight from (X0, Y0) by
    (ddx, ddy) cells, by direct quadrature of the charge crossing each
    dual-cell face and of the time-averaged overlap with each node cell."""
    tau = (np.arange(nsub) + 0.5) / nsub
    Xc = X0 + tau * ddx
    Yc = Y0 + tau * ddy
    J = np.zeros((3, ny, nx))
    ilo, ihi = int(math.floor(min(X0, X0 + ddx))) - 2, int(math.floor(max(X0, X0 + ddx))) + 3
    jlo, jhi = int(math.floor(min(Y0, Y0 + ddy))) - 2, int(math.floor(max(Y0, Y0 + ddy))) + 3

    def overlap(c, a):  # length of [c-1/2, c+1/2] inside [a-1/2, a+1/2]
        return np.clip(np.minimum(c + 0.5, a + 0.5) - np.maximum(c - 0.5, a - 0.5), 0.0, None)

    for i in range(ilo, ihi):
        for j in range(jlo, jhi):
            # face x = i + 1/2, y in [j-1/2, j+1/2]  (Jx[i, j])
            inside = np.abs(Xc - (i + 0.5)) < 0.5
            J[0, j % ny, i % nx] += q * ddx * np.mean(inside * overlap(Yc, j)) * dx / dt
            # face y = j + 1/2, x in [i-1/2, i+1/2]  (Jy[i, j])
            inside = np.abs(Yc - (j + 0.5)) < 0.5
            J[1, j % ny, i % nx] += q * ddy * np.mean(inside * overlap(Xc, i)) * dy / dt
            # out-of-plane current at node (i, j): q vz times mean overlap area
            J[2, j % ny, i % nx] += q * vz * np.mean(overlap(Xc, i) * overlap(Yc, j))
    return J


def new_position(nx, ny, ix, iy, x, y, ddx, ddy):
    X = ix + x + ddx
    Y = iy + y + ddy
    return X % nx, Y % ny


# ---------------------------------------------------------------- interpolation
def test_interp_reproduces_bilinear_functions(ora):
    """Bilinear interpolation is exact for span{1, X, Y, XY} sampled at each
    component's staggered points (Sec. 3.1, linear interpolation)."""
    nx, ny = 16, 12
    rng = np.random.default_rng(11)
    coef = rng.uniform(-1, 1, size=(6, 4))
    I, Jg = np.meshgrid(np.arange(nx), np.arange(ny))
    F = np.zeros((6, ny, nx))
    for c, (sx, sy) in enumerate(STAGGER):
        X, Y = I + sx, Jg + sy
        a, b, cc, d = coef[c]
        F[c] = a + b * X + cc * Y + d * X * Y
    for _ in range(200):
        ix, iy = rng.integers(2, nx - 3), rng.integers(2, ny - 3)
        x, y = rng.random(), rng.random()
        out = ora.interp(nx, ny, F[:3], F[3:], ix, iy, x, y)
        X, Y = ix + x, iy + y
        want = coef[:, 0] + coef[:, 1] * X + coef[:, 2] * Y + coef[:, 3] * X * Y
        np.testing.assert_allclose(out, want, rtol=0, atol=1e-12)


def test_interp_constant_field_everywhere(ora):
    nx, ny = 8, 8
    E = np.array([1.5, -2.0, 0.25])[:, None, None] * np.ones((3, ny, nx))
    B = np.array([-0.5, 3.0, 7.0])[:, None, None] * np.ones((3, ny, nx))
    for ix, iy, x, y in [(0, 0, 0.0, 0.0), (7, 7, 0.999, 0.999), (0, 7, 0.01, 0.6), (3, 4, 0.5, 0.5)]:
        out = ora.interp(nx, ny, E, B, ix, iy, x, y)
        np.testing.assert_allclose(out, [1.5, -2.0, 0.25, -0.5, 3.0, 7.0], atol=1e-14)


# ---------------------------------------------------------------- Boris
def test_boris_pure_electric_kick(ora):
    """With B = 0, Eqs. (6)-(9) reduce to u += (q/m) E dt."""
    rng = np.random.default_rng(1)
    for _ in range(100):
        qm, dt = rng.choice([-1.0, 1.0, -0.01]), 0.07
        E = rng.normal(size=3)
        u = rng.normal(size=3)
        out = ora.boris(qm, dt, np.r_[E, 0, 0, 0], u)
        np.testing.assert_allclose(out, u + qm * E * dt, rtol=0, atol=1e-14)


def test_boris_pure_magnetic_rotation(ora):
    """With E = 0 the update is a rotation about B: |u| and u.B are kept, the
    angle is 2 atan(|q/m| |B| dt / (2 gamma)), and the sense is that of
    du/dt = (q/m) u/gamma x B (Eq. 2)."""
    rng = np.random.default_rng(2)
    for _ in range(200):
        qm = rng.choice([-1.0, 1.0, -3.0])
        dt = 0.07
        B = rng.normal(size=3) * rng.uniform(0.1, 5)
        u = rng.normal(size=3) * rng.uniform(0.01, 3)
        out = ora.boris(qm, dt, np.r_[0, 0, 0, B], u)
        assert abs(np.linalg.norm(out) - np.linalg.norm(u)) <= 4e-16 * np.linalg.norm(u) * 8
        bh = B / np.linalg.norm(B)
        assert abs(out @ bh - u @ bh) < 1e-13 * np.linalg.norm(u)
        up0, up1 = u - (u @ bh) * bh, out - (out @ bh) * bh
        gamma = math.sqrt(1 + u @ u)
        theta = 2 * math.atan(abs(qm) * np.linalg.norm(B) * dt / (2 * gamma))
        cosang = up0 @ up1 / (np.linalg.norm(up0) * np.linalg.norm(up1))
        sinang = np.cross(up0, up1) @ bh / (np.linalg.norm(up0) * np.linalg.norm(up1))
        ang = math.atan2(sinang, cosang)
        assert abs(abs(ang) - theta) < 1e-12
        # sense: first-order step is along (q/m) (u x B)
        force = qm * np.cross(u, B)
        assert np.sign(ang) == np.sign(np.cross(up0, force) @ bh)


def _rotate(v, axis, ang):
    """v rotated about the unit vector axis by ang (right-handed; Rodrigues)."""
    return v * math.cos(ang) + np.cross(axis, v) * math.sin(ang) + axis * (axis @ v) * (1 - math.cos(ang))


def test_boris_parallel_electric_and_magnetic_fields(ora):
    """E parallel to B, both non-zero: the parallel momentum gains exactly
    (q/m) E dt, the perpendicular momentum keeps its length and turns by
    2 atan(|q/m| |B| dt / (2 gamma-)), gamma- being the Lorentz factor after
    the first half kick u- = u + (q/m) E dt / 2 (the reading of Eq. 10).

    What fails if the oracle is wrong:
      * gamma taken from u instead of u-: the angle check (the kick here
        changes gamma by 5-60 %);
      * one full E kick after the rotation (or before it) instead of the
        two half kicks of Eqs. (6) and (9): the angle check (the rotation
        then sees gamma(u) or gamma(u + (q/m) E dt));
      * a wrong sign or a dropped factor in either kick: the parallel check."""
    rng = np.random.default_rng(21)
    for _ in range(200):
        qm = rng.choice([-1.0, 1.0, -2.0])
        dt = 0.07
        bh = rng.normal(size=3)
        bh /= np.linalg.norm(bh)
        Bm = rng.uniform(0.5, 20.0)
        Em = rng.choice([-1.0, 1.0]) * rng.uniform(2.0, 20.0)
        u = rng.normal(size=3) * rng.uniform(0.05, 1.0)
        out = ora.boris(qm, dt, np.r_[Em * bh, Bm * bh], u)
        # parallel component: the two half kicks, nothing from the rotation
        assert abs(out @ bh - (u @ bh + qm * Em * dt)) < 1e-13 * (1 + abs(u @ bh))
        up0, up1 = u - (u @ bh) * bh, out - (out @ bh) * bh
        assert abs(np.linalg.norm(up1) - np.linalg.norm(up0)) < 1e-14 * (1 + np.linalg.norm(up0))
        um = u + 0.5 * qm * Em * dt * bh
        gm = math.sqrt(1 + um @ um)
        theta = 2 * math.atan(abs(qm) * Bm * dt / (2 * gm))
        # the sense of du/dt = (q/m) u/gamma x B is a rotation about -sign(q/m) B
        want = _rotate(up0, -np.sign(qm) * bh, theta)
        np.testing.assert_allclose(up1, want, rtol=0, atol=1e-13 * (1 + np.linalg.norm(up0)))


def test_boris_solves_the_time_centred_equation(ora):
    """General E and B, both non-zero: the Boris update (Eqs. 6-10) is the
    exact solution of the implicit, time-centred form of Eq. (4) with the
    Lorentz factor held at gamma- (the reading of Eq. 10),

        u' - u = (q/m) dt [E + (u' + u) / (2 gamma-) x B],
        gamma- = sqrt(1 + |u + (q/m) E dt / 2|^2),

    a 3 x 3 linear system for u' solved here with numpy.  Every arithmetic
    slip in the explicit sequence (a dropped half kick, gamma of u instead of
    u-, a sign in either cross product, s = t instead of 2t / (1 + t^2))
    breaks the equality."""
    rng = np.random.default_rng(22)
    for _ in range(300):
        qm = rng.choice([-1.0, 1.0, -0.01, 3.0])
        dt = 0.07
        E = rng.normal(size=3) * rng.uniform(0.1, 20.0)
        B = rng.normal(size=3) * rng.uniform(0.1, 20.0)
        u = rng.normal(size=3) * rng.uniform(0.01, 3.0)
        out = ora.boris(qm, dt, np.r_[E, B], u)
        a = qm * dt
        um = u + 0.5 * a * E
        k = a / (2 * math.sqrt(1 + um @ um))
        # u' - k u' x B = u + aE + k u x B, with u' x B = -[B]x u'
        Bx = np.array([[0, -B[2], B[1]], [B[2], 0, -B[0]], [-B[1], B[0], 0]])
        want = np.linalg.solve(np.eye(3) + k * Bx, u + a * E + k * np.cross(u, B))
        np.testing.assert_allclose(out, want, rtol=0, atol=1e-12 * (1 + np.linalg.norm(want)))


def test_boris_keeps_the_exb_drift(ora):
    """Crossed E and B (|E| < |B|): a particle whose momentum is gamma- v_E,
    v_E = E x B / |B|^2 the drift velocity, feels no net force
    (E + v_E x B = 0) and keeps its momentum; any other perpendicular momentum
    w = u - gamma- v_E turns rigidly about B (the drift frame).  gamma- is
    that of u- = u + (q/m) E dt / 2; for u = gamma- v_E it has the closed
    form |u|^2 = (1 + (q/m)^2 E^2 dt^2 / 4) |v_E|^2 / (1 - |v_E|^2).
    gamma of u instead of u-, or a single full E kick, leaves a residual
    force and fails the first check."""
    rng = np.random.default_rng(23)
    for _ in range(200):
        qm = rng.choice([-1.0, 1.0])
        dt = 0.07
        bh = rng.normal(size=3)
        bh /= np.linalg.norm(bh)
        eh = np.cross(bh, rng.normal(size=3))
        eh /= np.linalg.norm(eh)
        Bm = rng.uniform(1.0, 10.0)
        Em = Bm * rng.uniform(0.05, 0.9)
        E, B = Em * eh, Bm * bh
        vE = np.cross(E, B) / (Bm * Bm)
        h2 = (0.5 * qm * Em * dt) ** 2
        umag = math.sqrt((1 + h2) * (vE @ vE) / (1 - vE @ vE))
        u = umag * vE / np.linalg.norm(vE)
        out = ora.boris(qm, dt, np.r_[E, B], u)
        np.testing.assert_allclose(out, u, rtol=0, atol=1e-13 * (1 + umag))
        # add a perpendicular offset w and a parallel momentum p: in the drift
        # frame w turns by 2 atan(|q/m| B dt / (2 gamma-)), p is untouched
        w = np.cross(bh, eh) * rng.uniform(-1, 1) + eh * rng.uniform(-1, 1)
        p = rng.uniform(-1, 1)
        u2 = u + w + p * bh
        um = u2 + 0.5 * qm * dt * E
        gm = math.sqrt(1 + um @ um)
        out2 = ora.boris(qm, dt, np.r_[E, B], u2)
        theta = 2 * math.atan(abs(qm) * Bm * dt / (2 * gm))
        drift = gm * vE
        want = drift + _rotate(u2 - drift - p * bh, -np.sign(qm) * bh, theta) + p * bh
        np.testing.assert_allclose(out2, want, rtol=0, atol=1e-12 * (1 + np.linalg.norm(want)))


def test_cyclotron_orbit_radius(ora):
    """Uniform B_z, full particle advance (interp + Boris + Eq. 11): the
    positions are the vertices of a regular polygon whose circumradius is
    r_L sqrt(1 + eps^2), eps = |q/m| B dt / (2 gamma)."""
    nx = ny = 64
    dx = dy = 0.1
    dt = 0.07
    Bz = 2.0
    E = np.zeros((3, ny, nx))
    B = np.zeros((3, ny, nx))
    B[2] = Bz
    u0 = np.array([0.3, 0.0, 0.1])
    sp = ora.OracleSpecies(-1.0, -1.0, [30], [30], [0.25], [0.5], [u0[0]], [u0[1]], [u0[2]])
    sim = ora.OracleSim(nx, ny, dx, dy, dt, [sp], E, B)
    pts = []
    for _ in range(400):
        sim.push_deposit()
        pts.append(((sp.ix[0] + sp.x[0]) * dx, (sp.iy[0] + sp.y[0]) * dy))
    P = np.array(pts)
    # algebraic circle fit
    A = np.c_[2 * P[:, 0], 2 * P[:, 1], np.ones(len(P))]
    b = (P ** 2).sum(1)
    cx, cy, c = np.linalg.lstsq(A, b, rcond=None)[0]
    R = math.sqrt(c + cx * cx + cy * cy)
    gamma = math.sqrt(1 + u0 @ u0)
    rL = math.hypot(u0[0], u0[1]) / Bz
    eps = Bz * dt / (2 * gamma)
    assert abs(R / (rL * math.sqrt(1 + eps * eps)) - 1) < 1e-9
    np.testing.assert_allclose(np.hypot(P[:, 0] - cx, P[:, 1] - cy), R, rtol=1e-9)
    # momentum magnitude and u_z untouched by the rotation
    assert abs(math.hypot(sp.ux[0], sp.uy[0]) - 0.3) < 1e-13
    assert sp.uz[0] == 0.1


def test_free_streaming(ora):
    """E = B = 0: momenta stay bit-identical, X_n = X_0 + n v dt (mod L)."""
    nx, ny = 16, 8
    dx, dy, dt = 0.1, 0.2, 0.07
    rng = np.random.default_rng(3)
    n = 500
    ix = rng.integers(0, nx, n)
    iy = rng.integers(0, ny, n)
    x, y = rng.random(n), rng.random(n)
    u = rng.normal(size=(3, n)) * 0.7
    sp = ora.OracleSpecies(-1.0, -0.1, ix, iy, x, y, *u)
    sim = ora.OracleSim(nx, ny, dx, dy, dt, [sp])
    steps = 50
    for _ in range(steps):
        sim.push_deposit()
    assert np.array_equal(sp.ux, u[0]) and np.array_equal(sp.uy, u[1]) and np.array_equal(sp.uz, u[2])
    g = np.sqrt(1 + (u ** 2).sum(0))
    Xw = (ix + x + steps * u[0] / g * dt / dx) % nx
    Yw = (iy + y + steps * u[1] / g * dt / dy) % ny
    dXp = (sp.ix + sp.x - Xw + nx / 2) % nx - nx / 2
    dYp = (sp.iy + sp.y - Yw + ny / 2) % ny - ny / 2
    assert np.abs(dXp).max() < 1e-11 and np.abs(dYp).max() < 1e-11
    assert (sp.x >= 0).all() and (sp.x < 1).all() and (sp.y >= 0).all() and (sp.y < 1).all()


# ---------------------------------------------------------------- current deposit
def _deposit_cases(rng, n_random=300):
    cases = []
    for _ in range(n_random):
        cases.append((rng.integers(0, 6), rng.integers(0, 6), rng.random(), rng.random(),
                      rng.uniform(-0.99, 0.99), rng.uniform(-0.99, 0.99)))
    # forced: no crossing, x only, y only, both (x first / y first), corner hit,
    # exact face landing, zero motion, negative directions, grid-edge wrap
    cases += [
        (2, 2, 0.5, 0.5, 0.2, -0.1),
        (2, 2, 0.9, 0.5, 0.3, 0.05),
        (2, 2, 0.5, 0.1, 0.05, -0.3),
        (2, 2, 0.9, 0.8, 0.5, 0.25),
        (2, 2, 0.8, 0.9, 0.25, 0.5),
        (2, 2, 0.75, 0.75, 0.5, 0.5),     # hits the corner exactly
        (2, 2, 0.25, 0.25, -0.5, -0.5),
        (2, 2, 0.5, 0.5, 0.5, 0.0),       # lands exactly on x = 1
        (2, 2, 0.5, 0.5, 0.0, 0.0),
        (2, 2, 0.1, 0.2, -0.6, -0.7),
        (0, 0, 0.05, 0.05, -0.5, -0.4),   # wraps at the low edges
        (5, 5, 0.95, 0.95, 0.6, 0.7),     # wraps at the high edges
    ]
    return cases


def test_deposit_continuity_single_particle(ora):
    """Charge conservation, Eq. (12): rho(new) - rho(old) + dt div J = 0 for
    every 1-, 2- and 3-piece motion, with rho the node charge of the cloud."""
    nx, ny, dx, dy, dt, q = 6, 6, 0.1, 0.1, 0.07, -0.37
    rng = np.random.default_rng(4)
    for ix, iy, x, y, ddx, ddy in _deposit_cases(rng):
        J = ora.deposit_move(nx, ny, dx, dy, dt, q, 0.3, ix, iy, x, y, ddx, ddy)
        X1, Y1 = new_position(nx, ny, ix, iy, x, y, ddx, ddy)
        r0 = node_charge(nx, ny, q, ix + x, iy + y)
        r1 = node_charge(nx, ny, q, X1, Y1)
        res = r1 - r0 + dt * div_edge(J, dx, dy)
        assert np.abs(res).max() < 1e-13, (ix, iy, x, y, ddx, ddy)
        # total fluxes: the whole charge moved by (ddx, ddy) cells
        assert abs(J[0].sum() * dt / dx - q * ddx) < 1e-14
        assert abs(J[1].sum() * dt / dy - q * ddy) < 1e-14
        assert abs(J[2].sum() - q * 0.3) < 1e-14


def test_deposit_matches_brute_force_area_flux(ora):
    """Villasenor-Buneman fluxes (Eqs. 13-16 + splits) against a direct
    quadrature of the charge of the unit-square cloud crossing each face, and
    Jz against the time-averaged cloud/node-cell overlap."""
    nx, ny, dx, dy, dt, q, vz = 8, 8, 0.1, 0.1, 0.07, 0.5, -0.4
    rng = np.random.default_rng(5)
    cases = _deposit_cases(rng, n_random=12)
    for ix, iy, x, y, ddx, ddy in cases:
        ix, iy = ix + 1, iy + 1
        J = ora.deposit_move(nx, ny, dx, dy, dt, q, vz, ix, iy, x, y, ddx, ddy)
        Jb = brute_current(nx, ny, dx, dy, dt, q, vz, ix + x, iy + y, ddx, ddy)
        scale = abs(q) * dx / dt
        np.testing.assert_allclose(J[0], Jb[0], atol=2e-5 * scale)
        np.testing.assert_allclose(J[1], Jb[1], atol=2e-5 * scale)
        np.testing.assert_allclose(J[2], Jb[2], atol=1e-8)


def test_deposit_jz_reduces_to_cic_without_inplane_motion(ora):
    nx, ny = 6, 6
    J = ora.deposit_move(nx, ny, 0.1, 0.1, 0.07, 0.25, 0.6, 2, 3, 0.3, 0.8, 0.0, 0.0)
    want = node_charge(nx, ny, 0.25 * 0.6, 2.3, 3.8)
    np.testing.assert_allclose(J[2], want, atol=1e-15)
    assert np.abs(J[:2]).max() == 0.0


# ---------------------------------------------------------------- Yee solver
def _yee_mode_run(ora, mode, steps=200):
    nx, ny, dx, dy, dt = 32, 16, 0.1, 0.1, 0.07
    kx, ky = 2 * math.pi * 2 / (nx * dx), 2 * math.pi * 1 / (ny * dy)
    K2 = (2 * math.sin(kx * dx / 2) / dx) ** 2 + (2 * math.sin(ky * dy / 2) / dy) ** 2
    w = 2 / dt * math.asin(dt * math.sqrt(K2) / 2)
    I, Jg = np.meshgrid(np.arange(nx), np.arange(ny))
    E = np.zeros((3, ny, nx))
    B = np.zeros((3, ny, nx))
    J = np.zeros((3, ny, nx))
    if mode == "TM":   # Ez at the nodes
        f0 = np.cos(kx * I * dx + ky * Jg * dy)
        E[2] = f0
    else:              # Bz at the cell centres
        f0 = np.cos(kx * (I + 0.5) * dx + ky * (Jg + 0.5) * dy)
        B[2] = f0
    for n in range(1, steps + 1):
        ora.yee_b(nx, ny, dx, dy, dt / 2, E, B)
        ora.yee_e(nx, ny, dx, dy, dt, B, J, E)
        ora.yee_b(nx, ny, dx, dy, dt / 2, E, B)
        f = E[2] if mode == "TM" else B[2]
        np.testing.assert_allclose(f, f0 * math.cos(n * w * dt), atol=1e-11)
    return E, B, dx, dy


def test_yee_tm_mode_follows_discrete_dispersion(ora):
    """A single vacuum mode oscillates at (sin(w dt/2)/dt)^2 = sum_i (sin(k_i dx_i/2)/dx_i)^2,
    and div B stays zero (Eqs. 18-20, three-step update of Listing 3.1)."""
    E, B, dx, dy = _yee_mode_run(ora, "TM")
    divB = (np.roll(B[0], -1, axis=1) - B[0]) / dx + (np.roll(B[1], -1, axis=0) - B[1]) / dy
    assert np.abs(divB).max() < 1e-11


def test_yee_te_mode_follows_discrete_dispersion(ora):
    E, B, dx, dy = _yee_mode_run(ora, "TE")
    assert np.abs(div_edge(E, dx, dy)).max() < 1e-10


# ---------------------------------------------------------------- whole-step invariants
def _thermal_sim(ora, nx=16, ny=16, ppc=(2, 2), u_th=0.25, seed=7, fields=False):
    import pic_workloads as pw
    spec = pw.SpeciesSpec(-1.0, ppc, (u_th,) * 3, (0.05, -0.03, 0.0))
    st = pw.species_state(nx, ny, 4, spec, seed)
    sp = ora.OracleSpecies(spec.qm, spec.q, st["ix"], st["iy"], st["x"], st["y"], st["ux"], st["uy"], st["uz"])
    E = B = None
    if fields:
        E, B = pw.random_fields(nx, ny, 0.05, seed)
    return ora.OracleSim(nx, ny, 0.1, 0.1, 0.07, [sp], E, B)


def test_gauss_law_residual_is_preserved(ora):
    """div E - rho is constant in time to round-off: exact continuity of the
    deposit (Eq. 12) + Ampere's law on the Yee grid (Eqs. 17, 20)."""
    sim = _thermal_sim(ora, fields=True)
    s = sim.species[0]
    g0 = div_edge(sim.E, sim.dx, sim.dy) - node_charge(sim.nx, sim.ny, s.q, s.ix + s.x, s.iy + s.y)
    for _ in range(15):
        sim.push_deposit()
        sim.field_advance()
    g = div_edge(sim.E, sim.dx, sim.dy) - node_charge(sim.nx, sim.ny, s.q, s.ix + s.x, s.iy + s.y)
    assert np.abs(g - g0).max() < 1e-11


def test_langmuir_frequency_leapfrog(ora):
    """Cold plasma oscillation: w = (2/dt) asin(w_p dt / 2) (leapfrog), w_p = 1
    for unit density electrons; kinetic and field energy trade one-to-one."""
    import pic_workloads as pw
    nx, ny, dx, dy, dt = 512, 2, 0.1, 0.1, 0.07
    spec = pw.SpeciesSpec(-1.0, (4, 1), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    st = pw.species_state(nx, ny, 2, spec, 1)
    k = 2 * math.pi / (nx * dx)
    X = (st["ix"] + st["x"].astype(np.float64)) * dx
    v0 = 1e-4
    ux = v0 * np.sin(k * X)
    sp = ora.OracleSpecies(-1.0, spec.q, st["ix"], st["iy"], st["x"], st["y"], ux, 0 * ux, 0 * ux)
    sim = ora.OracleSim(nx, ny, dx, dy, dt, [sp])
    xs = (np.arange(nx) + 0.5) * dx
    amp, ue, uk = [], [], []
    for _ in range(500):
        uk_before = sim.energies()[2][0]          # u at t - dt/2
        sim.push_deposit()
        uk_after = sim.energies()[2][0]           # u at t + dt/2
        ue.append(sim.energies()[0])              # E at t (before the field update)
        uk.append(0.5 * (uk_before + uk_after))   # time-centred kinetic energy
        sim.field_advance()
        amp.append(sim.E[0, 0] @ np.sin(k * xs))   # Ex ~ sin(kx) for u_x ~ sin(kx)
    from scipy.optimize import curve_fit
    t = np.arange(1, 501) * dt
    a = np.array(amp)
    p, _ = curve_fit(lambda t, A, B, w: A * np.sin(w * t) + B * np.cos(w * t), t, a,
                     p0=[a[np.argmax(np.abs(a))], 0.0, 1.0])
    w_theory = 2 / dt * math.asin(dt / 2)
    assert abs(p[2] / w_theory - 1) < 5e-5, p[2] / w_theory
    assert abs(p[2] - 1.0) > 1.5e-4     # the leapfrog shift is resolved
    tot = np.array(ue) + np.array(uk)
    swing = np.ptp(ue)
    assert np.ptp(tot) < 5e-3 * swing


# ---------------------------------------------------------------- divergence diagnostics
def test_divergences_closed_form(ora):
    """The oracle's div E (at the nodes) and div B (at the cell centres) of
    single Fourier modes sampled at their staggered points equal the exact
    centred difference 2 sin(k d/2)/d times the mode at the divergence point."""
    nx, ny, dx, dy = 32, 24, 0.1, 0.2
    kx, ky = 2 * math.pi * 3 / (nx * dx), 2 * math.pi * 2 / (ny * dy)
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny))

    def sample(comp, f):
        sx, sy = STAGGER[comp]
        return f((ii + sx) * dx, (jj + sy) * dy)

    E = np.zeros((3, ny, nx))
    E[0] = sample(0, lambda X, Y: np.sin(kx * X))
    E[1] = sample(1, lambda X, Y: np.cos(ky * Y + 0.3))
    E[2] = 7.0                                     # Ez does not enter div E in 2D
    want = (2 * math.sin(kx * dx / 2) / dx * np.cos(kx * ii * dx)
            - 2 * math.sin(ky * dy / 2) / dy * np.sin(ky * jj * dy + 0.3))
    np.testing.assert_allclose(ora.div_e(nx, ny, dx, dy, E), want, atol=1e-11)

    B = np.zeros((3, ny, nx))
    B[0] = sample(3, lambda X, Y: np.cos(kx * X - 0.7))
    B[1] = sample(4, lambda X, Y: np.sin(ky * Y))
    B[2] = -5.0
    Xc, Yc = (ii + 0.5) * dx, (jj + 0.5) * dy
    want = (-2 * math.sin(kx * dx / 2) / dx * np.sin(kx * Xc - 0.7)
            + 2 * math.sin(ky * dy / 2) / dy * np.cos(ky * Yc))
    np.testing.assert_allclose(ora.div_b(nx, ny, dx, dy, B), want, atol=1e-11)


def test_divergence_of_yee_curl_vanishes(ora):
    """div B is unchanged by a Faraday half step from any E (div curl = 0 on the
    Yee grid), and div E is unchanged by an Ampere step with J = 0."""
    import pic_workloads as pw
    nx, ny, dx, dy = 24, 16, 0.1, 0.15
    E, B = pw.random_fields(nx, ny, 1.0, 11)
    E = E.astype(np.float64) + np.random.default_rng(3).standard_normal((3, ny, nx))
    B = B.astype(np.float64) + np.random.default_rng(4).standard_normal((3, ny, nx))
    d0 = ora.div_b(nx, ny, dx, dy, B)
    B2 = B.copy()
    ora.yee_b(nx, ny, dx, dy, 0.05, E, B2)
    assert np.abs(B2 - B).max() > 0.1
    np.testing.assert_allclose(ora.div_b(nx, ny, dx, dy, B2), d0, atol=1e-11)
    e0 = ora.div_e(nx, ny, dx, dy, E)
    E2 = E.copy()
    ora.yee_e(nx, ny, dx, dy, 0.05, B, np.zeros_like(B), E2)
    assert np.abs(E2 - E).max() > 0.1
    np.testing.assert_allclose(ora.div_e(nx, ny, dx, dy, E2), e0, atol=1e-11)


# ---------------------------------------------------------------- binomial current filter
def test_binomial_filter_fourier_response(ora):
    """Every periodic Fourier mode is an eigenvector of the binomial (1/4, 1/2,
    1/4) pass along x then y, with eigenvalue cos^2(pi m/nx) cos^2(pi l/ny);
    `passes` passes raise it to that power.  The Nyquist mode is removed, the
    mean is kept."""
    nx, ny = 24, 16
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny))
    for passes in (1, 2, 3):
        modes = [(1, 0, 0.3), (3, 5, -1.1), (nx // 2, 2, 0.0)]
        F = np.stack([np.cos(2 * math.pi * (m * ii / nx + l * jj / ny) + ph) for m, l, ph in modes])
        want = np.stack([(math.cos(math.pi * m / nx) ** 2 * math.cos(math.pi * l / ny) ** 2) ** passes * F[k]
                         for k, (m, l, _) in enumerate(modes)])
        ora.binomial_filter(nx, ny, passes, F)
        np.testing.assert_allclose(F, want, atol=1e-14)
    G = np.random.default_rng(5).standard_normal((ny, nx)) + 3.0
    s0 = G.sum()
    ora.binomial_filter(nx, ny, 4, G)
    assert abs(G.sum() - s0) < 1e-11


def test_filtered_current_keeps_continuity(ora):
    """The filter commutes with the discrete divergence, so the filtered current
    satisfies Eq. (12) exactly with the equally filtered charge density, and
    Gauss's law with it stays at its initial residual."""
    sim = _thermal_sim(ora, fields=True)
    sim.j_filter = 2
    s = sim.species[0]
    g0 = div_edge(sim.E, sim.dx, sim.dy) - sim.rho(filtered=True)
    for _ in range(3):
        r0 = sim.rho(filtered=True)
        raw0 = node_charge(sim.nx, sim.ny, s.q, s.ix + s.x, s.iy + s.y)
        sim.push_deposit()
        r1 = sim.rho(filtered=True)
        res = r1 - r0 + sim.dt * div_edge(sim.J, sim.dx, sim.dy)
        assert np.abs(res).max() < 1e-13 * np.abs(r1).max()
        # the plain node charge does not satisfy it with the filtered current
        raw1 = node_charge(sim.nx, sim.ny, s.q, s.ix + s.x, s.iy + s.y)
        assert np.abs(raw1 - raw0 + sim.dt * div_edge(sim.J, sim.dx, sim.dy)).max() > 1e-4 * np.abs(r1).max()
        sim.field_advance()
    g = div_edge(sim.E, sim.dx, sim.dy) - sim.rho(filtered=True)
    assert np.abs(g - g0).max() < 1e-11


# ---------------------------------------------------------------- Esirkepov deposit (variant)
def test_esirkepov_continuity_and_totals(ora):
    """Esirkepov's decomposition conserves charge exactly, Eq. (12), for every
    motion (the node charge of the cloud before and after, by overlap areas),
    and moves the whole charge: sum Jx dt/dx = q ddx, sum Jz = q vz."""
    nx, ny, dx, dy, dt, q, vz = 6, 6, 0.1, 0.1, 0.07, -0.37, 0.3
    rng = np.random.default_rng(14)
    for ix, iy, x, y, ddx, ddy in _deposit_cases(rng):
        J = ora.deposit_esirkepov(nx, ny, dx, dy, dt, q, vz, ix, iy, x, y, ddx, ddy)
        X1, Y1 = new_position(nx, ny, ix, iy, x, y, ddx, ddy)
        res = node_charge(nx, ny, q, X1, Y1) - node_charge(nx, ny, q, ix + x, iy + y) + dt * div_edge(J, dx, dy)
        assert np.abs(res).max() < 1e-13, (ix, iy, x, y, ddx, ddy)
        assert abs(J[0].sum() * dt / dx - q * ddx) < 1e-14
        assert abs(J[1].sum() * dt / dy - q * ddy) < 1e-14
        assert abs(J[2].sum() - q * vz) < 1e-14


def test_esirkepov_special_cases(ora):
    """(1) A motion that stays inside its cell: identical to the
    Villasenor-Buneman current (both reduce to the same linear-shape fluxes and
    the same time average for Jz).  (2) Motion along x only, crossing a face:
    the exact charge flux, checked by quadrature of the cloud.  (3) Motion
    along y only: no Jx.  (4) Exchanging x and y exchanges Jx and Jy and
    transposes the grid.  (5) An oblique crossing: a different current from
    the split Villasenor-Buneman one (the two schemes are not the same)."""
    nx, ny, dx, dy, dt, q, vz = 8, 8, 0.1, 0.1, 0.07, 0.5, -0.4
    rng = np.random.default_rng(15)
    for _ in range(200):
        x, y = rng.uniform(0.05, 0.95, 2)
        ddx = rng.uniform(-x, 1 - x) * 0.999
        ddy = rng.uniform(-y, 1 - y) * 0.999
        Je = ora.deposit_esirkepov(nx, ny, dx, dy, dt, q, vz, 3, 4, x, y, ddx, ddy)
        Jv = ora.deposit_move(nx, ny, dx, dy, dt, q, vz, 3, 4, x, y, ddx, ddy)
        np.testing.assert_allclose(Je, Jv, atol=1e-13)
    scale = abs(q) * dx / dt
    for x, y, ddx in ((0.8, 0.3, 0.45), (0.2, 0.7, -0.6), (0.5, 0.5, 0.5)):
        Je = ora.deposit_esirkepov(nx, ny, dx, dy, dt, q, vz, 3, 4, x, y, ddx, 0.0)
        Jb = brute_current(nx, ny, dx, dy, dt, q, vz, 3 + x, 4 + y, ddx, 0.0)
        np.testing.assert_allclose(Je[0], Jb[0], atol=2e-5 * scale)
        np.testing.assert_allclose(Je[1], 0.0, atol=1e-15)
    Je = ora.deposit_esirkepov(nx, ny, dx, dy, dt, q, vz, 3, 4, 0.4, 0.8, 0.0, 0.7)
    assert np.abs(Je[0]).max() == 0.0 and np.abs(Je[1]).max() > 0.1 * scale
    for x, y, ddx, ddy in ((0.9, 0.2, 0.3, 0.5), (0.1, 0.95, -0.4, 0.2), (0.7, 0.8, 0.6, 0.45)):
        A = ora.deposit_esirkepov(8, 6, dx, dx, dt, q, vz, 3, 2, x, y, ddx, ddy)
        Bt = ora.deposit_esirkepov(6, 8, dx, dx, dt, q, vz, 2, 3, y, x, ddy, ddx)
        np.testing.assert_allclose(A[0], Bt[1].T, atol=1e-14)
        np.testing.assert_allclose(A[1], Bt[0].T, atol=1e-14)
        np.testing.assert_allclose(A[2], Bt[2].T, atol=1e-14)
    Je = ora.deposit_esirkepov(nx, ny, dx, dy, dt, q, vz, 3, 4, 0.9, 0.8, 0.4, 0.5)
    Jv = ora.deposit_move(nx, ny, dx, dy, dt, q, vz, 3, 4, 0.9, 0.8, 0.4, 0.5)
    assert np.abs(Je[0] - Jv[0]).max() > 1e-3 * scale


def test_esirkepov_whole_step_gauss(ora):
    """Full steps with the Esirkepov deposit keep Gauss's law at its initial
    residual, like the split Villasenor-Buneman deposit."""
    sim = _thermal_sim(ora, fields=True)
    sim.esirkepov = True
    s = sim.species[0]
    g0 = div_edge(sim.E, sim.dx, sim.dy) - node_charge(sim.nx, sim.ny, s.q, s.ix + s.x, s.iy + s.y)
    for _ in range(10):
        sim.push_deposit()
        sim.field_advance()
    g = div_edge(sim.E, sim.dx, sim.dy) - node_charge(sim.nx, sim.ny, s.q, s.ix + s.x, s.iy + s.y)
    assert np.abs(g - g0).max() < 1e-11


# ---------------------------------------------------------------- moving window
def _lattice_column(nx, ny, ppc, column):
    px, py = ppc
    a, b, j = np.meshgrid(np.arange(px), np.arange(py), np.arange(ny), indexing="ij")
    n = a.size
    return {"ix": np.full(n, column, np.int32), "iy": j.reshape(-1).astype(np.int32),
            "x": ((a.reshape(-1) + 0.5) / px), "y": ((b.reshape(-1) + 0.5) / py),
            "ux": np.zeros(n), "uy": np.zeros(n), "uz": np.zeros(n)}


def test_moving_window_keeps_a_uniform_plasma(ora):
    """A window shift over a uniform cold lattice plasma, with a fresh lattice
    column injected at the new right edge, gives back the same plasma: the
    same number of particles, the same positions and exactly the same node
    charge."""
    import pic_workloads as pw
    nx, ny, T = 16, 8, 4
    spec = pw.SpeciesSpec(-1.0, (2, 2), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    st = pw.species_state(nx, ny, T, spec, 1)
    sp = ora.OracleSpecies(spec.qm, spec.q, st["ix"], st["iy"], st["x"], st["y"], st["ux"], st["uy"], st["uz"])
    sim = ora.OracleSim(nx, ny, 0.1, 0.1, 0.07, [sp])
    r0 = sim.rho()
    pos0 = sorted(zip(sp.ix.tolist(), sp.iy.tolist(), sp.x.tolist(), sp.y.tolist()))
    sim.move_window([_lattice_column(nx, ny, (2, 2), nx - 1)], T)
    s = sim.species[0]
    assert s.ix.size == st["ix"].size
    assert sorted(zip(s.ix.tolist(), s.iy.tolist(), s.x.tolist(), s.y.tolist())) == pos0
    np.testing.assert_array_equal(sim.rho(), r0)
    tiles = (s.iy // T) * (nx // T) + s.ix // T
    assert (np.diff(tiles) >= 0).all()          # re-sorted by tile


def test_moving_window_holds_a_light_pulse(ora):
    """A vacuum light pulse travelling in +x, with the window shifted by one
    cell whenever light has crossed one cell (every 2 steps at c dt = dx/2),
    stays where it is in window coordinates; without the shifts it moves
    about one cell per two steps."""
    nx, ny, dx, dt = 256, 4, 0.1, 0.05
    X = np.arange(nx)
    def pulse():
        E = np.zeros((3, ny, nx))
        B = np.zeros((3, ny, nx))
        E[2] = np.exp(-((X - 60.0) / 8.0) ** 2)[None, :]
        # By at (i + 1/2), a quarter cell behind: half a time step at c dt = dx / 2
        B[1] = -np.exp(-((X + 0.5 - 60.0 - 0.25) / 8.0) ** 2)[None, :]
        return E, B
    def centroid(E):
        w = E[2, 0] ** 2
        return (w * X).sum() / w.sum()
    for shift in (True, False):
        E, B = pulse()
        sim = ora.OracleSim(nx, ny, dx, dx, dt, [], E, B)
        c0 = centroid(sim.E)
        for n in range(1, 81):
            sim.push_deposit()
            sim.field_advance()
            if shift and n % 2 == 0:
                sim.move_window([], 4)
        moved = centroid(sim.E) - c0
        if shift:
            assert abs(moved) < 1.0, moved
        else:
            assert abs(moved - 40.0) < 1.0, moved


# ------------------------------------------------ valid initial fields (Eqs. 17-18)
def _curl_e(E, dx, dy):
    """z-curl of (Ex, Ey) at the cell centres, the Bz stencil of Eq. 19."""
    return (np.roll(E[1], -1, axis=1) - E[1]) / dx - (np.roll(E[0], -1, axis=0) - E[0]) / dy


def _curl_b(B, dx, dy):
    """z-curl of (Bx, By) at the nodes, the Ez stencil of Eq. 20."""
    return (B[1] - np.roll(B[1], 1, axis=1)) / dx - (B[0] - np.roll(B[0], 1, axis=0)) / dy


def _div_centre(B, dx, dy):
    """Divergence of (Bx, By) at the cell centres."""
    return (np.roll(B[0], -1, axis=1) - B[0]) / dx + (np.roll(B[1], -1, axis=0) - B[1]) / dy


@pytest.mark.parametrize("axis", [0, 1])
def test_solve_gauss_single_mode_closed_form(ora, axis):
    """A charge density cos(theta i) along one axis, E = 0 before: the discrete
    Gauss law gives E = A d / (2 sin(theta / 2)) sin(theta (i + 1/2)) along
    that axis and nothing along the other."""
    nx, ny, dx, dy, m, A = 48, 40, 0.1, 0.07, 3, 0.37
    n, d = (nx, dx) if axis == 0 else (ny, dy)
    th = 2 * np.pi * m / n
    prof = A * np.cos(th * np.arange(n))
    rho = np.tile(prof, (ny, 1)) if axis == 0 else np.tile(prof[:, None], (1, nx))
    E, B = np.zeros((3, ny, nx)), np.zeros((3, ny, nx))
    ora.solve_gauss(nx, ny, dx, dy, E, B, rho + 5.0)      # a uniform part changes nothing
    want = A * d / (2 * np.sin(th / 2)) * np.sin(th * (np.arange(n) + 0.5))
    got = E[0, 0, :] if axis == 0 else E[1, :, 0]
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * abs(want).max())
    assert np.abs(E[1 - axis]).max() < 1e-13 and np.abs(E[2]).max() == 0 and np.abs(B).max() == 0


def test_solve_gauss_random_fields(ora):
    """Random E, B and a random particle charge: afterwards div E = rho -
    <rho> at every node and div B = 0 at every cell centre (to round-off),
    while the discrete curls of E and B and the z components are unchanged."""
    import pic_workloads as pw
    nx, ny, dx, dy = 40, 56, 0.1, 0.12
    E, B = pw.random_fields(nx, ny, 0.3, 4)
    E, B = E.astype(np.float64), B.astype(np.float64)
    B[0] += np.random.default_rng(1).normal(0, 0.1, (ny, nx))   # give B a divergence
    rng = np.random.default_rng(2)
    n = 3000
    X, Y = rng.random(n) * nx, rng.random(n) * ny
    ix, iy = np.floor(X).astype(np.int32), np.floor(Y).astype(np.int32)
    rho = node_charge(nx, ny, -0.05, X, Y)
    assert np.allclose(rho, ora.rho(nx, ny, -0.05, ix, iy, X - ix, Y - iy))
    E0, B0 = E.copy(), B.copy()
    ora.solve_gauss(nx, ny, dx, dy, E, B, rho)
    res = div_edge(E, dx, dy) - (rho - rho.mean())
    assert np.abs(res).max() < 1e-11 * np.abs(rho).max()
    assert np.abs(_div_centre(B, dx, dy)).max() < 1e-11 * np.abs(B).max() / dx
    assert np.abs(_div_centre(B0, dx, dy)).max() > 0.1           # it had one
    np.testing.assert_allclose(_curl_e(E, dx, dy), _curl_e(E0, dx, dy), rtol=0, atol=1e-11)
    np.testing.assert_allclose(_curl_b(B, dx, dy), _curl_b(B0, dx, dy), rtol=0, atol=1e-11)
    assert np.array_equal(E[2], E0[2]) and np.array_equal(B[2], B0[2])
    # fields that already satisfy both laws are left as they are
    E1, B1 = E.copy(), B.copy()
    ora.solve_gauss(nx, ny, dx, dy, E1, B1, rho)
    assert np.abs(E1 - E).max() < 1e-12 and np.abs(B1 - B).max() < 1e-12


def test_solve_gauss_equals_the_one_dimensional_prefix_sum(ora):
    """The displaced Langmuir lattice: the projection from E = 0 reproduces
    the one-dimensional construction (running sum of rho - <rho> along x,
    zero mean)."""
    import sys, os
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    from langmuir_fixture import DX, langmuir_state
    nx, ny = 128, 16
    spec, st, E_ref = langmuir_state(nx, ny, 16)
    rho = ora.rho(nx, ny, spec.q, st["ix"], st["iy"], st["x"], st["y"])
    E, B = np.zeros((3, ny, nx)), np.zeros((3, ny, nx))
    ora.solve_gauss(nx, ny, DX, DX, E, B, rho)
    np.testing.assert_allclose(E, E_ref, rtol=0, atol=1e-12 * np.abs(E_ref).max())

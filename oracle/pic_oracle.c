/*
 * Plain FP64 CPU oracle for the 2D3V electromagnetic particle-in-cell step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference
 * that the HIP path is checked against.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header or
 * constant with the GPU library: it has no tiles, no guard cells and no LDS; it
 * indexes the periodic grid modulo (nx, ny) and walks the particles one by one
 * in array order, following the serial loop of the paper (Sec. 3.2, Listing 3.1).
 *
 * Conventions (normalised units of Eqs. 21-22, so c = 1):
 *   - A particle lives in cell (ix, iy) with in-cell offsets x, y in [0, 1);
 *     its position in cell units is X = ix + x, Y = iy + y.  Node (i, j) sits at
 *     the integer point (i, j).
 *   - Yee staggering (Fig. 3.1 is lost; standard 2D layout):
 *       Ex (i+1/2, j)   Ey (i, j+1/2)   Ez (i, j)
 *       Bx (i, j+1/2)   By (i+1/2, j)   Bz (i+1/2, j+1/2)
 *     J is co-located with E, the charge density with the nodes.
 *   - A field array holds three components, each an (ny x nx) row-major plane:
 *     F[c*nx*ny + j*nx + i].
 *   - q is the charge carried by one macro-particle (a charge density, e.g.
 *     -n0/ppc), qm the species charge-to-mass ratio.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IDX(i, j, nx) ((int64_t)(j) * (nx) + (i))

static int wrap(int i, int n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

/* ------------------------------------------------------------------------ */
/* Field interpolation (Sec. 3.1: linear interpolation from the cell and its  */
/* neighbours on the staggered grid).                                         */
/* ------------------------------------------------------------------------ */

/* Bilinear interpolation of one staggered component sampled at (i+sx, j+sy). */
static double interp_component(const double *F, int nx, int ny, double X,
                               double Y, double sx, double sy)
{
    double xs = X - sx, ys = Y - sy;
    double fi = floor(xs), fj = floor(ys);
    double wx = xs - fi, wy = ys - fj;
    int i0 = (int)fi, j0 = (int)fj;
    double v = 0.0;
    for (int b = 0; b < 2; b++)
        for (int a = 0; a < 2; a++) {
            double w = (a ? wx : 1.0 - wx) * (b ? wy : 1.0 - wy);
            v += w * F[IDX(wrap(i0 + a, nx), wrap(j0 + b, ny), nx)];
        }
    return v;
}

/* Stagger offsets of the six field components, in the order Ex Ey Ez Bx By Bz. */
static const double STAG_X[6] = {0.5, 0.0, 0.0, 0.0, 0.5, 0.5};
static const double STAG_Y[6] = {0.0, 0.5, 0.0, 0.5, 0.0, 0.5};

/* E and B at a particle: out = {Ex, Ey, Ez, Bx, By, Bz}. */
void ora_interp(int nx, int ny, const double *E, const double *B, int ix,
                int iy, double x, double y, double *out)
{
    const int64_t plane = (int64_t)nx * ny;
    double X = ix + x, Y = iy + y;
    for (int c = 0; c < 3; c++) {
        out[c] = interp_component(E + c * plane, nx, ny, X, Y, STAG_X[c],
                                  STAG_Y[c]);
        out[3 + c] = interp_component(B + c * plane, nx, ny, X, Y,
                                      STAG_X[3 + c], STAG_Y[3 + c]);
    }
}

/* ------------------------------------------------------------------------ */
/* Relativistic Boris push, Eqs. (6)-(10).                                    */
/* ------------------------------------------------------------------------ */

static void cross(const double a[3], const double b[3], double out[3])
{
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

/*
 * u holds u(t - dt/2) on entry and u(t + dt/2) on exit.  EB = {E, B} at the
 * particle at time t.  The rotation vector n of Eq. (10) uses the Lorentz
 * factor of u- (Eq. 6), which equals that of u+ since Eqs. (7)-(8) are a pure
 * rotation.
 */
void ora_boris(double qm, double dt, const double *EB, double *u)
{
    const double h = 0.5 * qm * dt; /* q dt / 2m */
    double um[3], up[3], upl[3], n[3], s[3], c[3];
    for (int k = 0; k < 3; k++) um[k] = u[k] + h * EB[k]; /* Eq. (6) */
    double g = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    for (int k = 0; k < 3; k++) n[k] = (h / g) * EB[3 + k]; /* Eq. (10) */
    cross(um, n, c);
    for (int k = 0; k < 3; k++) up[k] = um[k] + c[k]; /* Eq. (7) */
    double nn = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
    for (int k = 0; k < 3; k++) s[k] = 2.0 * n[k] / (1.0 + nn);
    cross(up, s, c);
    for (int k = 0; k < 3; k++) upl[k] = um[k] + c[k]; /* Eq. (8) */
    for (int k = 0; k < 3; k++) u[k] = upl[k] + h * EB[k]; /* Eq. (9) */
}

/* ------------------------------------------------------------------------ */
/* Villasenor-Buneman charge-conserving current deposit, Eqs. (12)-(16),      */
/* with the split of a motion that crosses cell faces into 1, 2 or 3 pieces   */
/* that each stay inside one cell (Sec. 3.1, Figs. 3.4-3.5).                  */
/* ------------------------------------------------------------------------ */

static double clamp01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

/*
 * One piece of the motion, inside cell (cx, cy), from (xa, ya) to (xb, yb) in
 * that cell's frame ([0,1]^2), lasting the fraction frac of the time step.
 *
 * The particle is a unit square of charge q centred on its position.  With the
 * cloud inside cell (cx, cy) it straddles the dual-cell face x = cx + 1/2, and
 * the part of its height below y = cy + 1/2 is 1 - y: moving by dxk it pushes
 * q dxk (1 - y_mid) across face (cx+1/2, cy) and q dxk y_mid across
 * (cx+1/2, cy+1) (Eqs. 13-14 measured from the cell centre, y' = y - 1/2).
 * Eqs. (15)-(16) give Jy the same way.  Fluxes become current densities by
 * multiplying with dx/dt (dy/dt).
 *
 * The out-of-plane current has no flux form; it is deposited as q vz times
 * the exact time average, along the piece, of the bilinear weight of each
 * corner node.
 */
static void deposit_piece(int nx, int ny, double dx, double dy, double dt,
                          double *J, double q, double vz, int cx, int cy,
                          double xa, double ya, double xb, double yb,
                          double frac)
{
    const int64_t plane = (int64_t)nx * ny;
    double *Jx = J, *Jy = J + plane, *Jz = J + 2 * plane;
    double dxk = xb - xa, dyk = yb - ya;
    double xm = 0.5 * (xa + xb), ym = 0.5 * (ya + yb);
    int i0 = wrap(cx, nx), i1 = wrap(cx + 1, nx);
    int j0 = wrap(cy, ny), j1 = wrap(cy + 1, ny);

    Jx[IDX(i0, j0, nx)] += q * dxk * (1.0 - ym) * dx / dt;
    Jx[IDX(i0, j1, nx)] += q * dxk * ym * dx / dt;
    Jy[IDX(i0, j0, nx)] += q * dyk * (1.0 - xm) * dy / dt;
    Jy[IDX(i1, j0, nx)] += q * dyk * xm * dy / dt;

    for (int b = 0; b < 2; b++)
        for (int a = 0; a < 2; a++) {
            double f0 = a ? xa : 1.0 - xa, f1 = a ? xb : 1.0 - xb;
            double g0 = b ? ya : 1.0 - ya, g1 = b ? yb : 1.0 - yb;
            /* integral over s in [0,1] of (f0 + s(f1-f0)) (g0 + s(g1-g0)) */
            double w = (f0 * g0 + f1 * g1) / 3.0 + (f0 * g1 + f1 * g0) / 6.0;
            Jz[IDX(a ? i1 : i0, b ? j1 : j0, nx)] += q * vz * frac * w;
        }
}

/*
 * Deposit the current of a straight motion from offset (x, y) in cell (ix, iy)
 * by (ddx, ddy) cells, |ddx|, |ddy| < 1.  The path is cut where it meets the
 * faces x = 0 / x = 1 and y = 0 / y = 1 of the starting cell; the cut times,
 * in increasing order, give 1, 2 or 3 pieces.  Each piece lies inside the cell
 * that holds its midpoint.
 */
void ora_deposit_move(int nx, int ny, double dx, double dy, double dt,
                      double q, double vz, int ix, int iy, double x, double y,
                      double ddx, double ddy, double *J)
{
    double tau[4];
    int nt = 0;
    double x1 = x + ddx, y1 = y + ddy;
    tau[nt++] = 0.0;
    if (x1 >= 1.0) tau[nt++] = (1.0 - x) / ddx;
    else if (x1 < 0.0) tau[nt++] = -x / ddx;
    if (y1 >= 1.0) tau[nt++] = (1.0 - y) / ddy;
    else if (y1 < 0.0) tau[nt++] = -y / ddy;
    tau[nt++] = 1.0;
    if (nt == 4 && tau[2] < tau[1]) {
        double t = tau[1];
        tau[1] = tau[2];
        tau[2] = t;
    }
    for (int k = 0; k + 1 < nt; k++) {
        double ta = clamp01(tau[k]), tb = clamp01(tau[k + 1]);
        double xa = x + ta * ddx, ya = y + ta * ddy;
        double xb = x + tb * ddx, yb = y + tb * ddy;
        int cx = (int)floor(0.5 * (xa + xb));
        int cy = (int)floor(0.5 * (ya + yb));
        deposit_piece(nx, ny, dx, dy, dt, J, q, vz, ix + cx, iy + cy,
                      clamp01(xa - cx), clamp01(ya - cy), clamp01(xb - cx),
                      clamp01(yb - cy), tb - ta);
    }
}

/* ------------------------------------------------------------------------ */
/* Esirkepov's charge-conserving current (Esirkepov, Comput. Phys. Commun.   */
/* 135 (2001) 144), the alternative deposit to Eqs. (13)-(16) with splits:    */
/* the change of the particle's shape-function product over the step is      */
/* decomposed into an x part W^x and a y part W^y, and the current is their  */
/* running sum across the stencil.  Linear (cloud-in-cell) shape, and the    */
/* quadratic B-spline, with which the field gather weights the three nearest */
/* sample points of each component too (a higher-order extension of the      */
/* linear weighting of Sec. 3.1, not in the paper).                          */
/* ------------------------------------------------------------------------ */

/* Cloud-in-cell weight of a node at distance d (cells). */
static double shape_cic(double d)
{
    double a = fabs(d);
    return a < 1.0 ? 1.0 - a : 0.0;
}

/* Quadratic B-spline weight of a node at distance d (cells): the linear shape
 * convolved once more with the unit cell, three nodes wide. */
static double shape_quad(double d)
{
    double a = fabs(d);
    if (a <= 0.5) return 0.75 - a * a;
    if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
    return 0.0;
}

/*
 * Current of a straight motion from offset (x, y) in cell (ix, iy) by
 * (ddx, ddy) cells, |ddx|, |ddy| < 1, on the n x n nodes ix+lo .. ix+lo+n-1
 * (likewise in y), wide enough to hold the shape before and after.  With S0,
 * S1 the node weights before and after and DS = S1 - S0:
 *   W^x_kl = DSx_k (S0y_l + DSy_l / 2),   W^y_kl = DSy_l (S0x_k + DSx_k / 2),
 *   W^z_kl = S0x_k S0y_l + (DSx_k S0y_l + S0x_k DSy_l) / 2 + DSx_k DSy_l / 3,
 * and Jx at (k + 1/2, l) = -q dx/dt sum_{k' <= k} W^x_k'l (likewise Jy),
 * Jz at (k, l) = q vz W^z_kl.
 */
static void esirkepov(int nx, int ny, double dx, double dy, double dt, double q,
                      double vz, int ix, int iy, double x, double y, double ddx,
                      double ddy, double *J, double (*shape)(double), int lo,
                      int n)
{
    const int64_t plane = (int64_t)nx * ny;
    double *Jx = J, *Jy = J + plane, *Jz = J + 2 * plane;
    double s0x[6], s1x[6], dsx[6], s0y[6], s1y[6], dsy[6];
    for (int k = 0; k < n; k++) {
        double p = lo + k; /* node position relative to the starting cell */
        s0x[k] = shape(x - p);
        s1x[k] = shape(x + ddx - p);
        dsx[k] = s1x[k] - s0x[k];
        s0y[k] = shape(y - p);
        s1y[k] = shape(y + ddy - p);
        dsy[k] = s1y[k] - s0y[k];
    }
    for (int l = 0; l < n; l++) {
        int j = wrap(iy + lo + l, ny);
        double run = 0.0;
        for (int k = 0; k + 1 < n; k++) {
            run -= dsx[k] * (s0y[l] + 0.5 * dsy[l]);
            Jx[IDX(wrap(ix + lo + k, nx), j, nx)] += q * run * dx / dt;
        }
    }
    for (int k = 0; k < n; k++) {
        int i = wrap(ix + lo + k, nx);
        double run = 0.0;
        for (int l = 0; l + 1 < n; l++) {
            run -= dsy[l] * (s0x[k] + 0.5 * dsx[k]);
            Jy[IDX(i, wrap(iy + lo + l, ny), nx)] += q * run * dy / dt;
        }
    }
    for (int l = 0; l < n; l++)
        for (int k = 0; k < n; k++) {
            double w = s0x[k] * s0y[l] + 0.5 * (dsx[k] * s0y[l] + s0x[k] * dsy[l]) +
                       dsx[k] * dsy[l] / 3.0;
            Jz[IDX(wrap(ix + lo + k, nx), wrap(iy + lo + l, ny), nx)] += q * vz * w;
        }
}

/* Linear shape: the 4 x 4 nodes ix-1 .. ix+2 hold it before and after. */
void ora_deposit_esirkepov(int nx, int ny, double dx, double dy, double dt,
                           double q, double vz, int ix, int iy, double x,
                           double y, double ddx, double ddy, double *J)
{
    esirkepov(nx, ny, dx, dy, dt, q, vz, ix, iy, x, y, ddx, ddy, J, shape_cic, -1, 4);
}

/* Quadratic shape: a position in (-1, 2) relative to the cell has its three
 * nodes within ix-2 .. ix+3, so the 6 x 6 nodes there hold it before and
 * after. */
void ora_deposit_esirkepov_quad(int nx, int ny, double dx, double dy,
                                double dt, double q, double vz, int ix, int iy,
                                double x, double y, double ddx, double ddy,
                                double *J)
{
    esirkepov(nx, ny, dx, dy, dt, q, vz, ix, iy, x, y, ddx, ddy, J, shape_quad, -2, 6);
}

/* Quadratic-shape gather of one staggered component sampled at (i+sx, j+sy):
 * the three sample points nearest the particle on each axis, weighted by the
 * shape at their distance. */
static double interp_component_quad(const double *F, int nx, int ny, double X,
                                    double Y, double sx, double sy)
{
    double xs = X - sx, ys = Y - sy;
    int i0 = (int)floor(xs + 0.5), j0 = (int)floor(ys + 0.5);
    double v = 0.0;
    for (int b = -1; b <= 1; b++)
        for (int a = -1; a <= 1; a++) {
            double w = shape_quad(xs - (i0 + a)) * shape_quad(ys - (j0 + b));
            v += w * F[IDX(wrap(i0 + a, nx), wrap(j0 + b, ny), nx)];
        }
    return v;
}

/* E and B at a particle with the quadratic shape: out = {Ex, .., Bz}. */
void ora_interp_quad(int nx, int ny, const double *E, const double *B, int ix,
                     int iy, double x, double y, double *out)
{
    const int64_t plane = (int64_t)nx * ny;
    double X = ix + x, Y = iy + y;
    for (int c = 0; c < 3; c++) {
        out[c] = interp_component_quad(E + c * plane, nx, ny, X, Y, STAG_X[c],
                                       STAG_Y[c]);
        out[3 + c] = interp_component_quad(B + c * plane, nx, ny, X, Y,
                                           STAG_X[3 + c], STAG_Y[3 + c]);
    }
}

/* Move one offset coordinate by d cells and renormalise it into [0, 1). */
static void advance_coord(int *i, double *x, double d, int n)
{
    double v = *x + d;
    if (v >= 1.0) {
        v -= 1.0;
        *i += 1;
    } else if (v < 0.0) {
        v += 1.0;
        *i -= 1;
        if (v >= 1.0) { /* round-off put it exactly on the face */
            v = 0.0;
            *i += 1;
        }
    }
    *x = v;
    *i = wrap(*i, n);
}

/*
 * The particle half of one time step (Listing 3.1, the loop over particles):
 * for every particle in array order, interpolate E and B, Boris-push the
 * momentum, move the particle by Eq. (11) and deposit its current into J
 * (which the caller zeroes; contributions of all species add up) --
 * deposit = 0: Villasenor-Buneman with splits, 1: Esirkepov, 2: the quadratic
 * shape, for the gather and Esirkepov's deposit both.
 * Returns 0, or -1 if a particle would move one cell or more (Eq. 1 violated).
 */
int ora_advance(int nx, int ny, double dx, double dy, double dt, double qm,
                double q, int64_t n, int32_t *ix, int32_t *iy, double *x,
                double *y, double *ux, double *uy, double *uz, const double *E,
                const double *B, double *J, int deposit)
{
    for (int64_t p = 0; p < n; p++) {
        double EB[6], u[3] = {ux[p], uy[p], uz[p]};
        if (deposit == 2)
            ora_interp_quad(nx, ny, E, B, ix[p], iy[p], x[p], y[p], EB);
        else
            ora_interp(nx, ny, E, B, ix[p], iy[p], x[p], y[p], EB);
        ora_boris(qm, dt, EB, u);
        double g = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        double ddx = u[0] / g * dt / dx; /* Eq. (11), in cells */
        double ddy = u[1] / g * dt / dy;
        if (fabs(ddx) >= 1.0 || fabs(ddy) >= 1.0) return -1;
        if (deposit == 2)
            ora_deposit_esirkepov_quad(nx, ny, dx, dy, dt, q, u[2] / g, ix[p],
                                       iy[p], x[p], y[p], ddx, ddy, J);
        else if (deposit == 1)
            ora_deposit_esirkepov(nx, ny, dx, dy, dt, q, u[2] / g, ix[p], iy[p],
                                  x[p], y[p], ddx, ddy, J);
        else
            ora_deposit_move(nx, ny, dx, dy, dt, q, u[2] / g, ix[p], iy[p],
                             x[p], y[p], ddx, ddy, J);
        int i = ix[p], j = iy[p];
        double xx = x[p], yy = y[p];
        advance_coord(&i, &xx, ddx, nx);
        advance_coord(&j, &yy, ddy, ny);
        ix[p] = i;
        iy[p] = j;
        x[p] = xx;
        y[p] = yy;
        ux[p] = u[0];
        uy[p] = u[1];
        uz[p] = u[2];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Yee finite-difference field advance, Eqs. (19)-(20) (Sec. 3.1).            */
/* ------------------------------------------------------------------------ */

/* Faraday's law, B -= h curl E. */
void ora_yee_b(int nx, int ny, double dx, double dy, double h, const double *E,
               double *B)
{
    const int64_t plane = (int64_t)nx * ny;
    const double *Ex = E, *Ey = E + plane, *Ez = E + 2 * plane;
    double *Bx = B, *By = B + plane, *Bz = B + 2 * plane;
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            int ip = wrap(i + 1, nx), jp = wrap(j + 1, ny);
            int64_t k = IDX(i, j, nx);
            double dEz_dy = (Ez[IDX(i, jp, nx)] - Ez[k]) / dy;
            double dEz_dx = (Ez[IDX(ip, j, nx)] - Ez[k]) / dx;
            double dEy_dx = (Ey[IDX(ip, j, nx)] - Ey[k]) / dx;
            double dEx_dy = (Ex[IDX(i, jp, nx)] - Ex[k]) / dy;
            Bx[k] -= h * dEz_dy;
            By[k] += h * dEz_dx;
            Bz[k] -= h * (dEy_dx - dEx_dy);
        }
}

/* Ampere's law with the particle current, E += h (curl B - J). */
void ora_yee_e(int nx, int ny, double dx, double dy, double h, const double *B,
               const double *J, double *E)
{
    const int64_t plane = (int64_t)nx * ny;
    const double *Bx = B, *By = B + plane, *Bz = B + 2 * plane;
    double *Ex = E, *Ey = E + plane, *Ez = E + 2 * plane;
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            int im = wrap(i - 1, nx), jm = wrap(j - 1, ny);
            int64_t k = IDX(i, j, nx);
            double dBz_dy = (Bz[k] - Bz[IDX(i, jm, nx)]) / dy;
            double dBz_dx = (Bz[k] - Bz[IDX(im, j, nx)]) / dx;
            double dBy_dx = (By[k] - By[IDX(im, j, nx)]) / dx;
            double dBx_dy = (Bx[k] - Bx[IDX(i, jm, nx)]) / dy;
            Ex[k] += h * (dBz_dy - J[k]);
            Ey[k] += h * (-dBz_dx - J[plane + k]);
            Ez[k] += h * (dBy_dx - dBx_dy - J[2 * plane + k]);
        }
}

/* The three-step field advance of Listing 3.1: B half step, E full step, B half step. */
void ora_field_advance(int nx, int ny, double dx, double dy, double dt,
                       double *E, double *B, const double *J)
{
    ora_yee_b(nx, ny, dx, dy, 0.5 * dt, E, B);
    ora_yee_e(nx, ny, dx, dy, dt, B, J, E);
    ora_yee_b(nx, ny, dx, dy, 0.5 * dt, E, B);
}

/* ------------------------------------------------------------------------ */
/* Strict re-sort of particles by tile (Sec. 4.3, the bucket sort of Fig.   */
/* 4.5): tile_offset is recounted from the final positions, and every        */
/* particle whose slot is outside its tile's new section moves into a hole.  */
/* ------------------------------------------------------------------------ */

/*
 * Tiles are T x T cells, numbered row-major: t = (iy / T) * (nx / T) + ix / T.
 * Output: off[0 .. ntiles] (new tile_offset) and src[0 .. n'): the particle at
 * slot j after the sort is the one that was at slot src[j].
 *
 * The pairing of holes and movers is not fixed by the paper (it registers them
 * with atomics).  The canonical choice made here: holes are the non-staying
 * slots in ascending order (so they come grouped by section), movers are the
 * non-staying particles ordered by destination tile and, within one tile, by
 * ascending slot; the k-th hole receives the k-th mover.
 *
 * removed (NULL: none): particles with removed[i] != 0 belong to no tile (the
 * moving window drops them); they are not counted, their slots are holes, and
 * the array shrinks to n' = n - (removed particles) slots.  Particles appended
 * to the array (the window's new particles) are movers like any other.
 * *n_out = n'.  Returns 0, or -1 if a cell index is out of range.
 */
int ora_sort_canonical(int nx, int ny, int T, int64_t n, const int32_t *ix,
                       const int32_t *iy, const unsigned char *removed,
                       int64_t *off, int64_t *src, int64_t *n_out)
{
    const int ntx = nx / T, nty = ny / T;
    const int64_t ntiles = (int64_t)ntx * nty;
    int64_t *tile = malloc(sizeof(int64_t) * (n ? n : 1));
    int64_t *cnt = calloc(ntiles + 1, sizeof(int64_t));
    int64_t *mstart = calloc(ntiles + 1, sizeof(int64_t));
    int64_t *holes = malloc(sizeof(int64_t) * (n ? n : 1));
    int64_t *movers = malloc(sizeof(int64_t) * (n ? n : 1));
    char *stay = malloc(n ? n : 1);
    int rc = 0;

    /* step (1): count the particles per tile at their final position */
    for (int64_t i = 0; i < n; i++) {
        if (removed && removed[i]) {
            tile[i] = -1;
            continue;
        }
        if (ix[i] < 0 || ix[i] >= nx || iy[i] < 0 || iy[i] >= ny) {
            rc = -1;
            goto done;
        }
        tile[i] = (int64_t)(iy[i] / T) * ntx + ix[i] / T;
        cnt[tile[i]]++;
    }
    off[0] = 0;
    for (int64_t t = 0; t < ntiles; t++) off[t + 1] = off[t] + cnt[t];
    const int64_t n_new = off[ntiles];

    /* a particle stays iff its slot is inside its tile's new section */
    for (int64_t i = 0; i < n; i++)
        stay[i] = tile[i] >= 0 && i >= off[tile[i]] && i < off[tile[i] + 1];

    /* steps (2)-(4): holes (non-staying slots of the new array) in ascending
       order; movers (non-staying particles that still exist) grouped by
       destination tile */
    int64_t nh = 0;
    for (int64_t i = 0; i < n_new; i++)
        if (!stay[i]) holes[nh++] = i;
    memset(cnt, 0, sizeof(int64_t) * (ntiles + 1));
    for (int64_t i = 0; i < n; i++)
        if (tile[i] >= 0 && !stay[i]) cnt[tile[i]]++;
    for (int64_t t = 0; t < ntiles; t++) mstart[t + 1] = mstart[t] + cnt[t];
    for (int64_t i = 0; i < n; i++)
        if (tile[i] >= 0 && !stay[i]) movers[mstart[tile[i]]++] = i;

    /* step (5): move */
    for (int64_t j = 0; j < n_new; j++) src[j] = j;
    for (int64_t k = 0; k < nh; k++) src[holes[k]] = movers[k];
    *n_out = n_new;

done:
    free(tile);
    free(cnt);
    free(mstart);
    free(holes);
    free(movers);
    free(stay);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* The motion-class sort, the alternative Sec. 4.3 cites (after Germaschewski */
/* et al.): by the Courant condition of Eq. (1) a particle ends each step in  */
/* its own tile or one of the eight around it, so its motion falls into one   */
/* of nine classes, and the array is regrouped by new tile in one counting    */
/* pass keyed on the class.                                                   */
/* ------------------------------------------------------------------------ */

/* Step of a tile index from a to b on a periodic axis of m tiles: 0, +1 or
 * -1; +1 when m == 2 (both neighbours are the same tile); 2 if b is further
 * than one tile from a. */
static int tile_step(int a, int b, int m)
{
    int d = wrap(b - a, m);
    if (d == 0) return 0;
    if (d == 1) return 1;
    if (d == m - 1) return -1;
    return 2;
}

/*
 * Input: n particles in their tile sections before the sort -- slots
 * off_old[s] .. off_old[s+1]-1 hold the particles of tile s (tile_offset,
 * Sec. 4.1) -- and their cells (ix, iy) after the push.  The class of the
 * particle at a slot of section s that now lies in tile t is
 * (dty + 1) * 3 + (dtx + 1), with (dtx, dty) the step from s to t on the
 * periodic tile grid (tile_step).
 * Output: the particles ordered by (new tile, class, old slot): off[0 ..
 * ntiles] the new tile_offset, src[j] the old slot of the particle that ends
 * at slot j.  Returns 0, or -1 if a cell is out of range or further than one
 * tile from its section's tile.
 */
int ora_sort_motion_classes(int nx, int ny, int T, int64_t n, const int32_t *ix,
                            const int32_t *iy, const int64_t *off_old,
                            int64_t *off, int64_t *src)
{
    const int ntx = nx / T, nty = ny / T;
    const int64_t ntiles = (int64_t)ntx * nty;
    int64_t *key = malloc(sizeof(int64_t) * (n ? n : 1));
    int64_t *start = calloc(ntiles * 9 + 1, sizeof(int64_t));
    int rc = 0;

    for (int64_t s = 0; s < ntiles && rc == 0; s++) {
        const int sx = (int)(s % ntx), sy = (int)(s / ntx);
        for (int64_t i = off_old[s]; i < off_old[s + 1]; i++) {
            if (ix[i] < 0 || ix[i] >= nx || iy[i] < 0 || iy[i] >= ny) {
                rc = -1;
                break;
            }
            const int tx = ix[i] / T, ty = iy[i] / T;
            const int dtx = tile_step(sx, tx, ntx), dty = tile_step(sy, ty, nty);
            if (dtx == 2 || dty == 2) {
                rc = -1;
                break;
            }
            key[i] = ((int64_t)ty * ntx + tx) * 9 + (dty + 1) * 3 + (dtx + 1);
            start[key[i] + 1]++;
        }
    }
    if (rc == 0) {
        /* counting sort on the key, stable in the old slot order */
        for (int64_t k = 0; k < ntiles * 9; k++) start[k + 1] += start[k];
        for (int64_t t = 0; t <= ntiles; t++) off[t] = start[t * 9];
        for (int64_t i = 0; i < n; i++) src[start[key[i]]++] = i;
    }
    free(key);
    free(start);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Diagnostics.                                                               */
/* ------------------------------------------------------------------------ */

/* Charge density at the nodes: area (CIC) weighting of the unit-square cloud. */
void ora_deposit_rho(int nx, int ny, double q, int64_t n, const int32_t *ix,
                     const int32_t *iy, const double *x, const double *y,
                     double *rho)
{
    for (int64_t p = 0; p < n; p++) {
        int i0 = ix[p], j0 = iy[p];
        int i1 = wrap(i0 + 1, nx), j1 = wrap(j0 + 1, ny);
        rho[IDX(i0, j0, nx)] += q * (1.0 - x[p]) * (1.0 - y[p]);
        rho[IDX(i1, j0, nx)] += q * x[p] * (1.0 - y[p]);
        rho[IDX(i0, j1, nx)] += q * (1.0 - x[p]) * y[p];
        rho[IDX(i1, j1, nx)] += q * x[p] * y[p];
    }
}

/* Node charge density with the quadratic shape (the three nodes nearest the
 * particle on each axis). */
void ora_deposit_rho_quad(int nx, int ny, double q, int64_t n, const int32_t *ix,
                          const int32_t *iy, const double *x, const double *y,
                          double *rho)
{
    for (int64_t p = 0; p < n; p++) {
        double X = ix[p] + x[p], Y = iy[p] + y[p];
        int i0 = (int)floor(X + 0.5), j0 = (int)floor(Y + 0.5);
        for (int b = -1; b <= 1; b++)
            for (int a = -1; a <= 1; a++)
                rho[IDX(wrap(i0 + a, nx), wrap(j0 + b, ny), nx)] +=
                    q * shape_quad(X - (i0 + a)) * shape_quad(Y - (j0 + b));
    }
}

/* 1/2 dx dy sum of F^2 over the three components of a field. */
double ora_field_energy(int nx, int ny, double dx, double dy, const double *F)
{
    double s = 0.0;
    for (int64_t k = 0; k < 3 * (int64_t)nx * ny; k++) s += F[k] * F[k];
    return 0.5 * dx * dy * s;
}

/* Kinetic energy dx dy sum m_p (gamma - 1), with particle mass m_p = q / qm. */
double ora_kinetic_energy(double dx, double dy, double qm, double q, int64_t n,
                          const double *ux, const double *uy, const double *uz)
{
    double s = 0.0;
    for (int64_t p = 0; p < n; p++) {
        double u2 = ux[p] * ux[p] + uy[p] * uy[p] + uz[p] * uz[p];
        s += sqrt(1.0 + u2) - 1.0;
    }
    return dx * dy * (q / qm) * s;
}

/* Discrete divergence of an E-staggered field at the nodes. */
void ora_div_e(int nx, int ny, double dx, double dy, const double *F,
               double *out)
{
    const int64_t plane = (int64_t)nx * ny;
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            int im = wrap(i - 1, nx), jm = wrap(j - 1, ny);
            out[IDX(i, j, nx)] =
                (F[IDX(i, j, nx)] - F[IDX(im, j, nx)]) / dx +
                (F[plane + IDX(i, j, nx)] - F[plane + IDX(i, jm, nx)]) / dy;
        }
}

/* ------------------------------------------------------------------------ */
/* Binomial filter (Listing 3.1: the optional smoothing of J after            */
/* update_gc_add).  One pass smooths a plane with the three-point binomial    */
/* kernel (1/4, 1/2, 1/4) along x, then along y, periodically; `passes`       */
/* passes are applied in turn.  The same filter applied to the charge density */
/* keeps the continuity equation exact, since it commutes with the discrete   */
/* divergence.                                                                */
/* ------------------------------------------------------------------------ */
void ora_binomial_filter(int nx, int ny, int passes, int64_t planes, double *F)
{
    const int64_t plane = (int64_t)nx * ny;
    double *tmp = (double *)malloc((size_t)plane * sizeof(double));
    if (!tmp) return;
    for (int64_t c = 0; c < planes; c++) {
        double *A = F + c * plane;
        for (int p = 0; p < passes; p++) {
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++)
                    tmp[IDX(i, j, nx)] = 0.25 * A[IDX(wrap(i - 1, nx), j, nx)] +
                                         0.5 * A[IDX(i, j, nx)] +
                                         0.25 * A[IDX(wrap(i + 1, nx), j, nx)];
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++)
                    A[IDX(i, j, nx)] = 0.25 * tmp[IDX(i, wrap(j - 1, ny), nx)] +
                                       0.5 * tmp[IDX(i, j, nx)] +
                                       0.25 * tmp[IDX(i, wrap(j + 1, ny), nx)];
        }
    }
    free(tmp);
}

/* Discrete divergence of B at the cell centres (i+1/2, j+1/2). */
void ora_div_b(int nx, int ny, double dx, double dy, const double *B,
               double *out)
{
    const int64_t plane = (int64_t)nx * ny;
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            int ip = wrap(i + 1, nx), jp = wrap(j + 1, ny);
            out[IDX(i, j, nx)] =
                (B[IDX(ip, j, nx)] - B[IDX(i, j, nx)]) / dx +
                (B[plane + IDX(i, jp, nx)] - B[plane + IDX(i, j, nx)]) / dy;
        }
}

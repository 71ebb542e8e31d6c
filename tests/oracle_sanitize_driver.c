/*
 * Test driver: runs every function of the C oracle on small inputs and edge
 * cases (empty particle sets, offsets at 0 and just below 1, particles on
 * the periodic seam, one-tile grids, removal in the sort) so that a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer can check it for
 * out-of-bounds accesses, leaks and undefined behaviour.  Exits 0 when every
 * call returned as expected.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void ora_interp(int nx, int ny, const double *E, const double *B, int ix, int iy, double x, double y, double *out);
void ora_boris(double qm, double dt, const double *EB, double *u);
void ora_deposit_move(int nx, int ny, double dx, double dy, double dt, double q, double vz, int ix, int iy, double x,
                      double y, double ddx, double ddy, double *J);
void ora_deposit_esirkepov(int nx, int ny, double dx, double dy, double dt, double q, double vz, int ix, int iy,
                           double x, double y, double ddx, double ddy, double *J);
int ora_advance(int nx, int ny, double dx, double dy, double dt, double qm, double q, int64_t n, int32_t *ix,
                int32_t *iy, double *x, double *y, double *ux, double *uy, double *uz, const double *E,
                const double *B, double *J, int deposit);
void ora_interp_quad(int nx, int ny, const double *E, const double *B, int ix, int iy, double x, double y,
                     double *out);
void ora_deposit_esirkepov_quad(int nx, int ny, double dx, double dy, double dt, double q, double vz, int ix,
                                int iy, double x, double y, double ddx, double ddy, double *J);
void ora_deposit_rho_quad(int nx, int ny, double q, int64_t n, const int32_t *ix, const int32_t *iy,
                          const double *x, const double *y, double *rho);
void ora_field_advance(int nx, int ny, double dx, double dy, double dt, double *E, double *B, const double *J);
int ora_sort_canonical(int nx, int ny, int T, int64_t n, const int32_t *ix, const int32_t *iy,
                       const unsigned char *removed, int64_t *off, int64_t *src, int64_t *n_out);
void ora_deposit_rho(int nx, int ny, double q, int64_t n, const int32_t *ix, const int32_t *iy, const double *x,
                     const double *y, double *rho);
double ora_field_energy(int nx, int ny, double dx, double dy, const double *F);
double ora_kinetic_energy(double dx, double dy, double qm, double q, int64_t n, const double *ux, const double *uy,
                          const double *uz);
void ora_div_e(int nx, int ny, double dx, double dy, const double *F, double *out);
void ora_binomial_filter(int nx, int ny, int passes, int64_t planes, double *F);
void ora_div_b(int nx, int ny, double dx, double dy, const double *B, double *out);

static uint64_t rng_state = 88172645463325252ull;
static double urand(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static int fail(const char *what)
{
    fprintf(stderr, "oracle driver: %s\n", what);
    return 1;
}

static int run_grid(int nx, int ny, int T, int64_t n, int deposit)
{
    const int64_t P = (int64_t)nx * ny;
    const double dx = 0.1, dy = 0.1, dt = 0.07;
    double *E = calloc(3 * P, sizeof(double)), *B = calloc(3 * P, sizeof(double)), *J = calloc(3 * P, sizeof(double));
    double *rho = calloc(P, sizeof(double)), *div = calloc(P, sizeof(double));
    const int64_t m = n > 0 ? n : 1;
    int32_t *ix = malloc(m * sizeof(int32_t)), *iy = malloc(m * sizeof(int32_t));
    double *x = malloc(m * sizeof(double)), *y = malloc(m * sizeof(double));
    double *ux = malloc(m * sizeof(double)), *uy = malloc(m * sizeof(double)), *uz = malloc(m * sizeof(double));
    unsigned char *rm = malloc(m);
    const int ntiles = (nx / T) * (ny / T);
    int64_t *off = malloc((ntiles + 1) * sizeof(int64_t)), *src = malloc(m * sizeof(int64_t)), nout = 0;
    int rc = 0;
    if (!E || !B || !J || !rho || !div || !ix || !iy || !x || !y || !ux || !uy || !uz || !rm || !off || !src)
        return fail("allocation");
    for (int64_t k = 0; k < 3 * P; ++k) {
        E[k] = 0.05 * (urand() - 0.5);
        B[k] = 0.05 * (urand() - 0.5);
    }
    for (int64_t p = 0; p < n; ++p) {
        ix[p] = (int32_t)(urand() * nx);
        iy[p] = (int32_t)(urand() * ny);
        x[p] = urand();
        y[p] = urand();
        if (p % 7 == 0) x[p] = 0.0;                          /* on a face */
        if (p % 11 == 0) y[p] = nextafter(1.0, 0.0);         /* just below the next face */
        if (p % 13 == 0) ix[p] = nx - 1;                     /* on the periodic seam */
        if (p % 17 == 0) iy[p] = 0;
        ux[p] = 3.0 * (urand() - 0.5);
        uy[p] = 3.0 * (urand() - 0.5);
        uz[p] = 0.5 * (urand() - 0.5);
        rm[p] = (unsigned char)(p % 5 == 0);
    }
    double out[6], u[3] = {0.3, -0.2, 0.1}, EB[6] = {0.01, 0.02, 0.03, 0.1, -0.2, 0.3};
    ora_interp(nx, ny, E, B, nx - 1, ny - 1, 0.999, 0.0, out);
    ora_boris(-1.0, dt, EB, u);
    ora_deposit_move(nx, ny, dx, dy, dt, -0.1, 0.2, nx - 1, 0, 0.95, 0.02, 0.6, -0.5, J);
    ora_deposit_esirkepov(nx, ny, dx, dy, dt, -0.1, 0.2, 0, ny - 1, 0.01, 0.98, -0.6, 0.5, J);
    /* quadratic shape at both seams: the stencils reach two nodes out */
    ora_interp_quad(nx, ny, E, B, nx - 1, 0, 0.999, 0.0, out);
    ora_interp_quad(nx, ny, E, B, 0, ny - 1, 0.0, 0.999, out);
    ora_deposit_esirkepov_quad(nx, ny, dx, dy, dt, -0.1, 0.2, 0, ny - 1, 0.01, 0.98, -0.99, 0.99, J);
    ora_deposit_esirkepov_quad(nx, ny, dx, dy, dt, -0.1, 0.2, nx - 1, 0, 0.99, 0.01, 0.99, -0.99, J);
    if (ora_advance(nx, ny, dx, dy, dt, -1.0, -0.1, n, ix, iy, x, y, ux, uy, uz, E, B, J, deposit) != 0)
        rc |= fail("advance");
    ora_field_advance(nx, ny, dx, dy, dt, E, B, J);
    ora_deposit_rho(nx, ny, -0.1, n, ix, iy, x, y, rho);
    ora_deposit_rho_quad(nx, ny, -0.1, n, ix, iy, x, y, rho);
    ora_div_e(nx, ny, dx, dy, E, div);
    ora_div_b(nx, ny, dx, dy, B, div);
    (void)ora_field_energy(nx, ny, dx, dy, E);
    (void)ora_kinetic_energy(dx, dy, -1.0, -0.1, n, ux, uy, uz);
    for (int passes = 0; passes < 3; ++passes) ora_binomial_filter(nx, ny, passes, 3, J);
    if (ora_sort_canonical(nx, ny, T, n, ix, iy, NULL, off, src, &nout) != 0 || nout != n) rc |= fail("sort");
    if (ora_sort_canonical(nx, ny, T, n, ix, iy, rm, off, src, &nout) != 0 || nout > n) rc |= fail("sort removal");
    free(E); free(B); free(J); free(rho); free(div); free(ix); free(iy); free(x); free(y);
    free(ux); free(uy); free(uz); free(rm); free(off); free(src);
    return rc;
}

int main(void)
{
    int rc = 0;
    rc |= run_grid(32, 24, 8, 2000, 0);
    rc |= run_grid(32, 24, 8, 2000, 1);
    rc |= run_grid(16, 16, 16, 500, 0);   /* one tile: every neighbour is itself */
    rc |= run_grid(16, 8, 8, 0, 0);       /* no particles */
    rc |= run_grid(8, 8, 8, 1, 1);
    rc |= run_grid(32, 24, 8, 2000, 2);   /* the quadratic shape */
    rc |= run_grid(8, 8, 8, 1, 2);
    if (!rc) printf("oracle driver: ok\n");
    return rc;
}

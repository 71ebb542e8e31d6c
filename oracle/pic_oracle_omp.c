/*
 * The FP64 oracle's particle step and strict tile sort spread over the host's
 * cores with OpenMP -- the shape of the paper's CPU implementation (Sec.
 * 4.2.1): an OpenMP loop over the tiles, every thread advancing the particles
 * of its tiles with the serial oracle's own code (ora_advance) and depositing
 * their current into a private copy of J, the copies added into J afterwards.
 *
 * TEST INFRASTRUCTURE ONLY, like pic_oracle.c, whose functions it calls and
 * with which it is linked: it is the timed CPU baseline of the benchmark, not
 * a checker.  Its results equal the serial oracle's to FP64 round-off (the
 * current is summed in a different order); the sort is the same canonical
 * permutation, bit for bit.  Shares nothing with the GPU library.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int ora_advance(int nx, int ny, double dx, double dy, double dt, double qm,
                double q, int64_t n, int32_t *ix, int32_t *iy, double *x,
                double *y, double *ux, double *uy, double *uz, const double *E,
                const double *B, double *J, int esirkepov);

/* Threads the parallel regions below use. */
int ora_omp_threads(void) { return omp_get_max_threads(); }

/*
 * The particle half of a step for one species whose particles are grouped
 * by tile (tile t holds slots off[t] .. off[t+1]-1): every tile's particles
 * advanced by ora_advance into the calling thread's private current, the
 * private currents then added into J (which the caller zeroes; species add
 * up).  Returns 0, or -1 if a particle would move one cell or more.
 */
int ora_advance_omp(int nx, int ny, double dx, double dy, double dt, double qm,
                    double q, int64_t ntiles, const int64_t *off, int32_t *ix,
                    int32_t *iy, double *x, double *y, double *ux, double *uy,
                    double *uz, const double *E, const double *B, double *J)
{
    const int64_t len = 3 * (int64_t)nx * ny;
    const int nt = omp_get_max_threads();
    double *priv = calloc((size_t)nt * len, sizeof(double));
    int rc = 0;
    if (!priv) return -2;
#pragma omp parallel
    {
        double *Jp = priv + (int64_t)omp_get_thread_num() * len;
#pragma omp for schedule(dynamic, 4) reduction(| : rc)
        for (int64_t t = 0; t < ntiles; t++) {
            const int64_t a = off[t], n = off[t + 1] - off[t];
            if (n > 0 && ora_advance(nx, ny, dx, dy, dt, qm, q, n, ix + a, iy + a, x + a, y + a, ux + a,
                                     uy + a, uz + a, E, B, Jp, 0) != 0)
                rc |= 1;
        }
        /* J += sum of the private copies, each node by one thread, copies in
           thread order */
#pragma omp for schedule(static)
        for (int64_t k = 0; k < len; k++) {
            double s = J[k];
            for (int p = 0; p < nt; p++) s += priv[(int64_t)p * len + k];
            J[k] = s;
        }
    }
    free(priv);
    return rc ? -1 : 0;
}

/*
 * ora_sort_canonical's permutation (Sec. 4.3: holes in ascending order
 * filled by the movers ordered by destination tile, then by old slot),
 * computed with the work split over threads: the tile histogram, the stay
 * flags, the compaction of the holes and the counting sort of the movers by
 * destination tile all run on thread-sized chunks of the particle array,
 * whose partial counts are combined in chunk order.  Same inputs and outputs
 * as ora_sort_canonical without removed particles.
 */
int ora_sort_canonical_omp(int nx, int ny, int T, int64_t n, const int32_t *ix,
                           const int32_t *iy, int64_t *off, int64_t *src)
{
    const int ntx = nx / T, nty = ny / T;
    const int64_t ntiles = (int64_t)ntx * nty;
    const int nt = omp_get_max_threads();
    int64_t *tile = malloc(sizeof(int64_t) * (n ? n : 1));
    char *stay = malloc(n ? n : 1);
    int64_t *cnt = calloc((size_t)nt * ntiles, sizeof(int64_t));   /* [thread][tile] */
    int64_t *nhole = calloc((size_t)nt + 1, sizeof(int64_t));
    int64_t *holes = malloc(sizeof(int64_t) * (n ? n : 1));
    int rc = 0;
    if (!tile || !stay || !cnt || !nhole || !holes) {
        rc = -2;
        goto done;
    }
#pragma omp parallel reduction(| : rc)
    {
        const int me = omp_get_thread_num();
        const int64_t c0 = n * me / nt, c1 = n * (me + 1) / nt;
        int64_t *mine = cnt + (int64_t)me * ntiles;
        /* step (1): tile of every particle, histogram per chunk */
        for (int64_t i = c0; i < c1; i++) {
            if (ix[i] < 0 || ix[i] >= nx || iy[i] < 0 || iy[i] >= ny) {
                rc |= 1;
                tile[i] = 0;
                continue;
            }
            tile[i] = (int64_t)(iy[i] / T) * ntx + ix[i] / T;
            mine[tile[i]]++;
        }
#pragma omp barrier
#pragma omp single
        {
            off[0] = 0;
            for (int64_t t = 0; t < ntiles; t++) {
                int64_t s = 0;
                for (int p = 0; p < nt; p++) s += cnt[(int64_t)p * ntiles + t];
                off[t + 1] = off[t] + s;
            }
        }
        /* stay flags; holes of the chunk, ascending */
        int64_t h = 0;
        for (int64_t i = c0; i < c1; i++) {
            stay[i] = i >= off[tile[i]] && i < off[tile[i] + 1];
            h += !stay[i];
        }
        nhole[me + 1] = h;
        /* movers of the chunk per destination tile (the chunk's histogram is
           reused for them) */
        memset(mine, 0, sizeof(int64_t) * ntiles);
        for (int64_t i = c0; i < c1; i++)
            if (!stay[i]) mine[tile[i]]++;
#pragma omp barrier
#pragma omp single
        {
            for (int p = 0; p < nt; p++) nhole[p + 1] += nhole[p];
            /* movers' start per (tile, chunk): tiles ascending, chunks in order */
            int64_t run = 0;
            for (int64_t t = 0; t < ntiles; t++)
                for (int p = 0; p < nt; p++) {
                    const int64_t c = cnt[(int64_t)p * ntiles + t];
                    cnt[(int64_t)p * ntiles + t] = run;
                    run += c;
                }
        }
        int64_t hk = nhole[me];
        for (int64_t i = c0; i < c1; i++)
            if (!stay[i]) holes[hk++] = i;
#pragma omp barrier
        /* step (5): the k-th hole receives the k-th mover */
        for (int64_t i = c0; i < c1; i++) src[i] = i;
#pragma omp barrier
        for (int64_t i = c0; i < c1; i++)
            if (!stay[i]) src[holes[mine[tile[i]]++]] = i;
    }
done:
    free(tile);
    free(stay);
    free(cnt);
    free(nhole);
    free(holes);
    return rc ? -1 : 0;
}

/* Apply a sort's permutation to one species' arrays in place: element j
 * becomes the old element src[j] (the gather split over threads). */
int ora_permute_omp(int64_t n, const int64_t *src, int32_t *ix, int32_t *iy, double *x, double *y, double *ux,
                    double *uy, double *uz)
{
    int32_t *ti = malloc(sizeof(int32_t) * (n ? n : 1));
    double *td = malloc(sizeof(double) * (n ? n : 1));
    if (!ti || !td) {
        free(ti);
        free(td);
        return -2;
    }
    int32_t *iarr[2] = {ix, iy};
    double *darr[5] = {x, y, ux, uy, uz};
    for (int a = 0; a < 2; a++) {
        int32_t *v = iarr[a];
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < n; j++) ti[j] = v[src[j]];
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < n; j++) v[j] = ti[j];
    }
    for (int a = 0; a < 5; a++) {
        double *v = darr[a];
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < n; j++) td[j] = v[src[j]];
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < n; j++) v[j] = td[j];
    }
    free(ti);
    free(td);
    return 0;
}

// Internal declarations shared by the libpic translation units (host launchers
// and kernels).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pic.h"
#include "pic_push.h"

namespace pic {

struct SortSpecies {
    Parts p;              // the particle arrays (tile-relative cells)
    int32_t *gcell;       // the caller's cell array: whole-grid cells, written by the publish
    const LeaverRec *lrec;   // leaver particle data written by the push kernel
    Parts stg;            // the motion-class sort's staging, [n]: every particle at its new slot
    LeaverRec *srec;      // the in-place sort's mover staging, [n]: tile t's movers at off[t] + k, in hole order
    int32_t *off;         // tile_offset: the recount's first pass keeps it in offp and the scan
                          // writes the new one in its place
    int32_t *offp;        // the tile_offset before the sort (scratch)
    const int32_t *cnt;
    const uint32_t *leav;
    int32_t *hole;        // [n]: tile t's holes, ascending, at off[t] + k
    int32_t *mcount;      // [n_tiles]: movers (the motion-class sort: [3][n_tiles] class bases)
    int32_t *fcount;      // [n_tiles]: holes whose fill is pending (the next push fills them), else 0
    int32_t *fbase;       // [n_tiles][W]: first pending hole of each push wavefront's run
    int32_t *bsum;        // [n_tiles / kScanBlock + 1] block totals of the tile scan
    int32_t n;            // particles before the sort
    // moving window (else null / 0): new particles appended at slots
    // [n, n + inj_n), grouped by tile (tile t's at n + inj_off[t] ..), and a
    // device count of the particles that left
    const int32_t *inj_off;
    int32_t inj_n;
    const int32_t *removed;
};

struct SortArgs {
    int *err;
    int nx, ny, ntx, nty, tile;
    int n_tiles;
    int n_species;
    int defer;            // 1: the scatter leaves the holes to the next push (pic_step); the
                          // motion-class sort leaves its copy back to it, and sets *stg_live
    int *stg_live;        // nonzero: the particles wait in the motion-class sort's staging arrays
    int rebase;           // 1: no push since the last sort (the moving window's sort): cells are
                          // relative to their tile modulo its edge
    SortSpecies sp[kMaxSpecies];
};


// one binomial filter pass: `planes` planes of nx x ny values (float or double)
struct FilterArgs {
    const void *src;
    void *dst;
    int nx, ny, planes;
};

struct FieldArgs {
    float *fld;           // the nine field planes
    const float *jtile;   // tile current halos folded into J by the E step, or null: J is input
    const float *bh;      // B after the step's first half step, formed by the push (three planes),
                          // or null: the field advance forms it in place
    int nx, ny, ntx, nty;
    float hdx, hdy;       // (dt/2)/dx, (dt/2)/dy  (B half steps)
    float dt, dtdx, dtdy; // E full step
};

// ---- launchers (each defined next to its kernels) ----
// halo: the pad H of cadence_ok (1 unless particles are sorted less often than every step)
// ppl: particles per lane per pass of the push loop (1, 2 or 4; ppl_ok)
// ms: the particles may wait in the motion-class sort's staging arrays
// (PushArgs::stg_live decides on the device; the default current and deposit only)
void launch_push_deposit(int tile, int replicas, int jmode, int dmode, int halo, int ppl, const PushArgs &a,
                         int n_tiles, bool ms, hipStream_t s);
void launch_j_reduce(int tile, int halo, const JReduceArgs &r, hipStream_t s);
// rebase: the pushes follow a sort (PushArgs::rebase of every member)
void launch_push_batch(int tile, int replicas, int jmode, int dmode, int halo, int ppl, const PushArgs *descs,
                       const int4 *items, int n_items, bool rebase, hipStream_t s);
void launch_j_reduce_batch(int tile, int halo, const JReduceArgs *descs, const int4 *items, int n_items,
                           hipStream_t s);
void launch_set_int(int *p, int v, hipStream_t s);
void launch_sort_scan(const SortArgs &a, int n_tiles, hipStream_t s);
void launch_sort_plan(const SortArgs &a, int n_tiles, hipStream_t s);
void launch_sort_scatter(const SortArgs &a, int n_tiles, hipStream_t s);
void launch_fill(const SortArgs &a, int n_tiles, hipStream_t s);
// the whole-grid cells of every particle into the caller's cell arrays
// (gcell); rebase: no push since the last sort
void launch_publish(const SortArgs &a, int n_tiles, bool rebase, hipStream_t s);
// tile-relative cells of n particles grouped by tile, inside their tiles
void launch_localize(const int32_t *cell, int16_t *lcell, int32_t n, int tile, hipStream_t s);

// Batched sort phases.  Work tables (int4 per block):
//   count/add: (sim, species, block of kScanBlock tiles)   scan: (sim, species)
//   plan/scatter: (sim, species, group of kSortWaves tiles)
struct SortBatch {
    const SortArgs *descs;
    const int4 *count_items; int n_count;
    const int4 *scan_items; int n_scan;
    const int4 *plan_items; int n_plan;
    int max_blocks;   // the most scan blocks of one member
};
// a pending hole fill of every member (fill_unit), and the publish of their cells
void launch_fill_batch(const SortBatch &b, hipStream_t s);
void launch_publish_batch(const SortBatch &b, bool rebase, hipStream_t s);
// motion: the motion-class sort (PIC_FLAG_MOTION_SORT) instead of the in-place one
void launch_sort_batch(const SortBatch &b, bool motion, hipStream_t s);
// the motion-class sort after the recount and scan: every particle into the
// staging arrays at its new slot, then the staging arrays copied back
void launch_motion_scatter(const SortArgs &a, int n_tiles, hipStream_t s);
void launch_motion_copy(const SortArgs &a, int n_tiles, hipStream_t s);
// the copy back only if *stg_live is set (a deferred one), then *stg_live = 0
void launch_motion_copy_live(const SortArgs &a, int n_tiles, hipStream_t s);
// tile_offset (off, n_tiles + 1) of n cells grouped by tile; sets kErrOrder
// for a cell outside the grid and kErrGroup if they are not grouped (off is
// then meaningless but every write stays inside it)
void launch_init_tiles(const int32_t *cell, int32_t n, int nx, int ny, int tile, int ntx, int n_tiles, int32_t *off,
                       int *err, hipStream_t s);
// grouping caller particles by tile: stable radix sort on the tile id
// (k_tilesort.hip), in place on p
struct TileSortArgs {
    GParts p;                    // n each: the particle arrays (the caller's, whole-grid cells)
    GParts tmp;                  // n each: a copy of them is made here
    uint32_t *key[2], *val[2];   // n each: double buffers
    int32_t *hist;               // tile_sort_hist_entries(n)
    int n, tile, ntx, n_tiles;
};
int64_t tile_sort_hist_entries(int n);
void launch_tile_sort(const TileSortArgs &a, hipStream_t s);
// the two phases: the permutation (radix passes; null if nothing to sort),
// then the gather of the particle arrays through tmp
const uint32_t *launch_tile_sort_perm(const TileSortArgs &a, hipStream_t s);
void launch_tile_sort_gather(const TileSortArgs &a, const uint32_t *perm, hipStream_t s);
// moving window (window column i lives in array column (i + origin) mod nx):
// E and B of array column col become zero
void launch_zero_column(float *fld, int nx, int ny, int col, hipStream_t s);
// p[0 .. n) = 0 (a kernel, not a memset node)
void launch_zero_i32(int32_t *p, int n, hipStream_t s);
// the particles of array column col leave; leaver sub-lists and count records
// of every tile in the push kernel's format (no leaver copies: a removed
// particle is nobody's mover)
struct WindowSpecies {
    Parts p;                     // tile-relative cells
    const int32_t *off;
    int32_t *cnt;
    uint32_t *leav;
    int32_t *removed;   // device count of the particles that left
};
void launch_window_remove(int tile, const WindowSpecies &w, int ntx, int nty, int n_tiles, int col, hipStream_t s);
// new particles given in window column nx - 1 into array column col (checked):
// whole-grid cells to dst, and cells relative to their tiles (of edge tile) to ldst
void launch_place_new(const int32_t *src, int32_t *dst, int16_t *ldst, int n, int nx, int ny, int col, int tile,
                      int *err, hipStream_t s);
void launch_filter(const FilterArgs &a, bool fp64, hipStream_t s);
void launch_filter_batch(const FilterArgs *descs, const int4 *items, int n_items, hipStream_t s);
// the three Yee sub-steps (k_field.hip); with f.jtile set, the E step folds
// the tile current halos (tiles of edge `tile`, halo pad `halo`) into J
void launch_field_advance(const FieldArgs &f, int tile, int halo, hipStream_t s);
// batched: items (simulation, 64 x 4 cell block); fold: every member's
// FieldArgs has jtile set
void launch_field_advance_batch(const FieldArgs *descs, const int4 *items, int n_items, bool fold, bool bh, int tile,
                                int halo, hipStream_t s);

// Conjugate-gradient projection of E (Eq. 17) or B (Eq. 18), k_poisson.hip.
constexpr int kCgPartials = 1024;   // per-block partial sums of one dot product, at most
struct CgScratch {
    double *x, *r, *p, *q;   // nx * ny each
    double *partial;         // kCgPartials
    double *scal;            // r.r (two parity slots), p.q, sum of the right-hand side
};
struct CgResult {
    int iterations;   // -1: a HIP call failed
    double residual;  // ||r|| / ||r0|| at the end
    bool converged;
};
CgResult cg_project(float *fld, const double *rho, double rho_bar, int magnetic, int nx, int ny, double dx, double dy,
                    double tol, int max_iter, const CgScratch &w, hipStream_t s);

struct DiagSpecies {
    const int32_t *cell;
    const float *x, *y, *ux, *uy, *uz;
    int32_t n;
    double q;
    int quadratic;   // the particle shape: 0 linear, 1 quadratic B-spline
};
void launch_diag_field_energy(const float *fld, int64_t plane, double *acc, hipStream_t s);
void launch_diag_kinetic(const DiagSpecies &sp, double *acc, hipStream_t s);
void launch_diag_rho(const DiagSpecies &sp, int nx, int ny, double *rho, hipStream_t s);
void launch_diag_continuity(const double *rho_prev, const double *rho_now, const float *J,
                            int nx, int ny, double dt, double dx, double dy, double *acc,
                            hipStream_t s);
void launch_diag_gauss(const float *fld, const double *rho, double rho_bar, int nx, int ny, double dx, double dy,
                       double *acc, hipStream_t s);
void launch_diag_counts(const int32_t *cnt, const int32_t *mcount, int n_tiles,
                        unsigned long long *acc, hipStream_t s);

}  // namespace pic

// Internal declarations shared by the libpic translation units (host launchers
// and kernels).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pic.h"

namespace pic {

constexpr int kMaxSpecies = PIC_MAX_SPECIES;
constexpr int kBlock = 256;          // threads per sort / stencil block (4 wavefronts)
constexpr int kSortWaves = kBlock / 64;   // tiles per sort plan / scatter block (one per wavefront)
constexpr int kCntStride = 32;       // ints per tile in the count record
constexpr int kScanBlock = 256;      // tiles per block of the tile-count scan

// Wavefronts that push one tile (one workgroup of 64 * W threads): 4 up to
// 16 x 16 tiles; 16 for 32 x 32 tiles, whose LDS (E/B halo and current) fills
// most of a compute unit, so a single workgroup must bring the occupancy.
__host__ __device__ constexpr int push_waves(int T) { return T >= 32 ? 16 : 4; }
constexpr int kMaxWaves = 16;

// Count record of one tile, written by the push kernel:
//   [0..8]        particles per direction of motion d = (dty+1)*3 + (dtx+1);
//                 [4] holds the particles that kept their tile
//   [9]           leavers (sum of the eight non-centre directions)
//   [10..10+W-1]  leavers found by wavefront w (length of leaver sub-list w)
constexpr int kCntLeavers = 9;
constexpr int kCntSub = 10;
// leaver-entry direction of a particle that left the moving window (no tile)
constexpr int kDirRemoved = 9;
static_assert(kCntSub + kMaxWaves <= kCntStride, "count record too short");

// Device error bits (ORed into Sim::err).
enum : int {
    kErrOrder = 1,   // particle outside its tile section / cell out of range
    kErrRange = 2,   // displacement of one cell or more
    kErrSort = 4,    // hole / mover count mismatch
    kErrCount = 8,   // tile counts do not sum to n
    kErrOverflow = 16, // a fixed-point current accumulator took 2^16 contributions or more
    kErrGroup = 32,  // caller particles not grouped by tile (cells in range)
};

// Current accumulation modes of the push kernel.
enum : int {
    kJFixed = 0,   // exact int64 fixed point in LDS (default)
    kJFloat = 1,   // FP32 LDS atomics, compensated replica sum
};

// Fixed-point resolution: one current contribution of the largest possible
// magnitude (the particle charge of the largest species times a full cell of
// motion) is 2^22 units; each contribution is rounded once to a unit
// (error at most 2^-23 of the largest one) and the sums are exact.
constexpr float kFixedScale = 4194304.0f;

// deposit scheme of the push kernel
constexpr int kDepVB = 0;          // Villasenor-Buneman with the 1/2/3-piece split (Eqs. 13-16)
constexpr int kDepEsirkepov = 1;   // Esirkepov's density decomposition (variant)

constexpr int kLdsBytes = 160 * 1024;   // LDS of one gfx950 compute unit
constexpr int kLeaverBuf = 64;           // leavers buffered per wavefront before a write-out
constexpr int kPieceBuf = 64;            // queued second / third motion pieces per wavefront
// one ballot can add a whole wavefront to either buffer
static_assert(kLeaverBuf >= 64 && kPieceBuf >= 64, "per-wavefront LDS buffers must hold 64 entries");

// Static LDS of the push kernel for tile T, R current replicas, mode JM and
// halo pad H (the sort cadence: between two sorts a particle may stray up to
// H - 1 cells outside its tile, so the E/B halo holds cells -H..T+H-1 and
// the current halo nodes -H..T+H).
constexpr int push_lds_bytes(int T, int R, int JM, int H = 1)
{
    return (T + 2 * H) * (T + 2 * H) * 48 + R * 3 * (T + 2 * H + 1) * (T + 2 * H + 1) * (JM == kJFixed ? 8 : 4) +
           kMaxSpecies * (9 + push_waves(T)) * 4 + push_waves(T) * 7 * kLeaverBuf * 4 +
           push_waves(T) * 6 * kPieceBuf * 4;
}

// Sort cadences the push kernel is built for: every 1, 2 or 4 steps, with
// the fixed-point current and one LDS copy of it when above 1.  A node's
// current halo then still overlaps at most one neighbour per axis (2H + 1 <=
// T), a position outside the tile has one periodic image within the pad
// (2H - 2 < T), and the LDS fits.
constexpr bool cadence_ok(int T, int H)
{
    return (H == 1 || H == 2 || H == 4) && 2 * H + 1 <= T && push_lds_bytes(T, 1, kJFixed, H) <= kLdsBytes;
}

// One species' particles as a structure of arrays (n entries each).
struct Parts {
    int32_t *cell;
    float *x, *y, *ux, *uy, *uz;
};

struct SpeciesDev {
    int32_t *cell;
    float *x, *y, *ux, *uy, *uz;
    const int32_t *off;   // tile_offset at the start of the step (n_tiles + 1)
    int32_t *cnt;         // [n_tiles][kCntStride]
    uint32_t *leav;       // [n]: leaver sub-lists, (slot - off[t]) << 4 | direction
    Parts lp;             // [n]: the leavers' new particle data, same positions as leav
    int32_t n;
    float h;              // (q/m) dt / 2
    float fq;             // charge in accumulator units: q / max|q| (x kFixedScale in fixed mode)
};

struct PushArgs {
    const float *fld;     // Ex Ey Ez Bx By Bz planes
    float *jtile;         // [n_tiles][3][(T+2H+1)^2], physical current of each tile halo
    int *err;
    int nx, ny, ntx, nty;
    float cx, cy;         // dt/dx, dt/dy
    float ju[3];          // accumulator unit -> physical Jx, Jy, Jz
    int n_species;
    SpeciesDev sp[kMaxSpecies];
};

// The part of a tile section [begin, end) streamed by wavefront w of the
// push kernel: the 64-aligned chunks covering the section are split into
// W contiguous runs.  Returns the slot range [lo, hi) (lo >= hi: none).
// The leavers found by wavefront w are stored from slot lo of the leaver list.
__host__ __device__ __forceinline__ void wave_range(int begin, int end, int w, int W, int &lo, int &hi)
{
    if (end <= begin) {
        lo = hi = begin;
        return;
    }
    const int c0 = begin >> 6, c1 = (end + 63) >> 6;
    const int q = (c1 - c0 + W - 1) / W;
    const int a = (c0 + w * q) << 6, b = (c0 + (w + 1) * q) << 6;
    lo = a > begin ? a : begin;
    hi = b < end ? b : end;
    if (hi < lo) hi = lo;
}

struct SortSpecies {
    Parts p;              // the particle arrays
    Parts lp;             // leaver particle data written by the push kernel
    Parts stg;            // mover staging, [n]: tile t's movers at offn[t] + k
    int32_t *off;         // tile_offset: read by the plan, replaced by the new one in the scatter
    int32_t *offn;        // new tile_offset (scratch)
    const int32_t *cnt;
    const uint32_t *leav;
    int32_t *hole;        // [n]: tile t's holes, ascending, at offn[t] + k
    int32_t *mcount;      // [n_tiles]
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
    SortSpecies sp[kMaxSpecies];
};

struct JReduceArgs {
    const float *jtile;
    float *J;             // the Jx plane; Jy, Jz follow
    int nx, ny, ntx, nty;
};

// one binomial filter pass: `planes` planes of nx x ny values (float or double)
struct FilterArgs {
    const void *src;
    void *dst;
    int nx, ny, planes;
};

struct FieldArgs {
    float *fld;
    int nx, ny;
    float hdx, hdy;       // (dt/2)/dx, (dt/2)/dy  (B half steps)
    float dt, dtdx, dtdy; // E full step
};

// ---- launchers (each defined next to its kernels) ----
// halo: the pad H of cadence_ok (1 unless particles are sorted less often than every step)
void launch_push_deposit(int tile, int replicas, int jmode, int dmode, int halo, const PushArgs &a, int n_tiles,
                         hipStream_t s);
void launch_j_reduce(int tile, int halo, const JReduceArgs &r, hipStream_t s);
void launch_push_batch(int tile, int replicas, int jmode, int dmode, int halo, const PushArgs *descs,
                       const int4 *items, int n_items, int *counter, int grid, hipStream_t s);
void launch_j_reduce_batch(int tile, int halo, const JReduceArgs *descs, const int4 *items, int n_items,
                           hipStream_t s);
void launch_set_int(int *p, int v, hipStream_t s);
void launch_sort_scan(const SortArgs &a, int n_tiles, hipStream_t s);
void launch_sort_plan(const SortArgs &a, int n_tiles, hipStream_t s);
void launch_sort_scatter(const SortArgs &a, int n_tiles, hipStream_t s);

// Batched sort phases.  Work tables (int4 per block):
//   count/add: (sim, species, block of kScanBlock tiles)   scan: (sim, species)
//   plan/scatter: (sim, species, group of kSortWaves tiles)
struct SortBatch {
    const SortArgs *descs;
    const int4 *count_items; int n_count;
    const int4 *scan_items; int n_scan;
    const int4 *plan_items; int n_plan;
};
void launch_sort_batch(const SortBatch &b, hipStream_t s);
// tile_offset (off, n_tiles + 1) of n cells grouped by tile; sets kErrOrder
// for a cell outside the grid and kErrGroup if they are not grouped (off is
// then meaningless but every write stays inside it)
void launch_init_tiles(const int32_t *cell, int32_t n, int nx, int ny, int tile, int ntx, int n_tiles, int32_t *off,
                       int *err, hipStream_t s);
// grouping caller particles by tile: stable radix sort on the tile id
// (k_tilesort.hip), in place on p
struct TileSortArgs {
    Parts p;                     // n each: the particle arrays
    Parts tmp;                   // n each: a copy of them is made here
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
    Parts p;
    const int32_t *off;
    int32_t *cnt;
    uint32_t *leav;
    int32_t *removed;   // device count of the particles that left
};
void launch_window_remove(int tile, const WindowSpecies &w, int ntx, int nty, int n_tiles, int col, hipStream_t s);
// new particles given in window column nx - 1 into array column col (checked)
void launch_place_new(const int32_t *src, int32_t *dst, int n, int nx, int ny, int col, int *err, hipStream_t s);
void launch_filter(const FilterArgs &a, bool fp64, hipStream_t s);
void launch_filter_batch(const FilterArgs *descs, const int4 *items, int n_items, hipStream_t s);
void launch_field_advance(const FieldArgs &f, hipStream_t s);
void launch_field_advance_batch(const FieldArgs *descs, const int4 *items, int n_items, hipStream_t s);

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

/*
 * libpic -- tiled 2D3V electromagnetic particle-in-cell step for AMD MI355X
 * (gfx950), C ABI.
 *
 * The library advances a periodic 2D plasma by the PIC cycle of Guidotti,
 * "Accelerating Particle-Mesh Algorithms with FPGAs and OmpSs@OpenCL":
 * per-tile field interpolation (Sec. 3.1), the relativistic Boris push
 * (Eqs. 6-10), the position advance (Eq. 11), Villasenor-Buneman
 * charge-conserving current deposition with cell-crossing splits
 * (Eqs. 12-16, Figs. 3.4-3.5), the strict re-sort of particles by tile
 * (Sec. 4.3), and the three-step Yee field update (Eqs. 19-20, Listing 3.1).
 *
 * Units are the normalised units of Eqs. (21)-(22): c = 1, charges in units
 * of e, masses in units of m_e, lengths in c / w_n, times in 1 / w_n.
 *
 * Memory model
 *   - Every device buffer is allocated and owned by the caller; the library
 *     keeps non-owning pointers and a small host-side record, and never frees
 *     caller memory.  pic_query() tells the caller what to allocate.
 *   - Every function that takes a hipStream_t enqueues its work on that stream
 *     and returns without synchronising, except pic_init(), pic_check(),
 *     pic_diag(), pic_get_state(), pic_set_state(), pic_get_tile_offsets()
 *     and pic_get_timing(), which synchronise the stream they are given.
 *   - Calls on one pic_sim must not run concurrently from several host
 *     threads.
 *   - The push and the sort keep each particle's cell in the workspace, as
 *     16 bits relative to its tile (the caller's cell array is read by
 *     pic_init and pic_set_state, and written back by pic_sync); x, y, ux, uy
 *     and uz they read and write in the caller's arrays.
 *   - pic_step() and pic_batch_step() leave the last part of their sort, the
 *     copy of the staged movers into their holes, to the next push, which
 *     streams those slots anyway: until then the particle arrays hold stale
 *     values in those slots.  With PIC_FLAG_MOTION_SORT, pic_step() likewise
 *     leaves the sorted particles in the workspace's staging arrays, where
 *     the next push reads them (the particle arrays hold the unsorted ones
 *     until then).  Every entry point that reads the particles
 *     (pic_get_state, pic_diag, pic_move_window, the Gauss solves, and of
 *     course the next push) completes it first.  A caller that reads the
 *     particle arrays itself calls pic_sync() before: it completes the fill
 *     and writes every particle's cell into the cell array.  tile_offset, the
 *     counts and the fields are final when pic_step() returns.
 *
 * Data layout
 *   - Grid: nx x ny cells, node (i, j) at (i dx, j dy), periodic in x and y.
 *     The field buffer holds nine FP32 planes of ny x nx values, row-major
 *     (index j * nx + i), in the order Ex Ey Ez Bx By Bz Jx Jy Jz.  Yee
 *     staggering: Ex and Jx at (i+1/2, j), Ey and Jy at (i, j+1/2), Ez and Jz
 *     at (i, j), Bx at (i, j+1/2), By at (i+1/2, j), Bz at (i+1/2, j+1/2).
 *   - Particles, one structure-of-arrays per species, n entries each:
 *       cell  int32  ix | (iy << 16), 0 <= ix < nx, 0 <= iy < ny
 *       x, y  float  offset inside the cell, in cells, in [0, 1)
 *       ux, uy, uz  float  momentum u = gamma v (Eq. 2)
 *     Particles are kept grouped by tile: tiles are tile x tile cells numbered
 *     row-major (t = (iy / tile) * (nx / tile) + ix / tile) and the particles
 *     of tile t occupy one contiguous section, sections in increasing t
 *     (pic_init and pic_set_state group particles given in any order).
 *     pic_sort() restores this order after every push (with sort_every = k
 *     > 1, after every k-th push: in between, a particle may be up to k - 1
 *     cells outside the tile whose section holds it).
 *
 * Errors: every int-returning call returns PIC_OK (0) or a negative PIC_E*
 * code; pic_strerror() names it.  Kernels that detect a bad state set a
 * device-side flag that pic_check() (and pic_diag()) read back.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_MAX_SPECIES 4

/* return codes */
#define PIC_OK 0
#define PIC_EINVAL (-1)   /* bad argument: sizes, pointers, alignment */
#define PIC_ECFL (-2)     /* dt violates the Courant condition, Eq. (1) */
#define PIC_ETILE (-3)    /* tile size unsupported or does not divide the grid */
#define PIC_EHIP (-4)     /* a HIP runtime call failed */
#define PIC_EORDER (-5)   /* particles not grouped by tile, or a cell out of range */
#define PIC_ERANGE (-6)   /* a particle tried to move one cell or more in a step */
#define PIC_ESORT (-7)    /* internal sort consistency check failed */
#define PIC_ECOUNT (-8)   /* tile counts do not add up to the particle count */
#define PIC_EOVERFLOW (-9) /* fixed-point current: a tile holds 2^31+ particles over all species */
#define PIC_ENOCONV (-10)  /* pic_solve_gauss: the iteration did not reach its tolerance */
#define PIC_ESCRATCH (-11) /* pic_solve_gauss_noalloc: grid larger than its static scratch holds */

/*
 * Current accumulation inside a tile (pic_config.flags).
 * Default (0): exact 64-bit fixed point -- each deposit contribution is the
 *   FP32 product of charge, motion and weight truncated to a unit of 2^-30 of
 *   the largest possible contribution (max |q| moving one cell, or at c for
 *   Jz), the sums are exact signed 64-bit integers, J is bit-reproducible
 *   from run to run and does not depend on the order of the additions.
 *   Limit: fewer than 2^31 particles in one tile over all species (else
 *   PIC_EOVERFLOW), which keeps every sum inside 64 bits.
 * PIC_FLAG_J_FLOAT: FP32 atomic adds into j_replicas LDS copies, summed with
 *   compensation; J reproducible only to round-off (and slower on gfx950).
 */
#define PIC_FLAG_J_FLOAT 1u

/*
 * Deposit scheme (pic_config.flags).  Default: Villasenor-Buneman fluxes
 * (Eqs. 13-16) of the 1, 2 or 3 pieces a motion is split into at cell faces
 * (Figs. 3.4-3.5).  PIC_FLAG_ESIRKEPOV: Esirkepov's density decomposition
 * (Comput. Phys. Commun. 135 (2001) 144) with the linear shape -- equal to the
 * default for motions inside one cell, a different charge-conserving current
 * on a 4 x 4 node stencil for motions that cross a face.  Fixed-point current
 * only (PIC_EINVAL together with PIC_FLAG_J_FLOAT).
 */
#define PIC_FLAG_ESIRKEPOV 2u

/*
 * Particle shape (pic_config.flags; not in the paper, which weights linearly,
 * Sec. 3.1): PIC_FLAG_QUADRATIC gives every particle the quadratic B-spline
 * shape, three nodes per axis.  The field gather weights the three nearest
 * sample points of each staggered component on each axis; the current is
 * Esirkepov's decomposition (as PIC_FLAG_ESIRKEPOV, which may be set too and
 * then changes nothing) with this shape, on the 4 x 4 nodes that hold the
 * shape before and after the motion; the charge density of pic_diag and
 * pic_solve_gauss uses it too.  The push stages a halo two cells wide and
 * carries one 64-particle chunk per lane.  Needs the fixed-point current,
 * j_replicas <= 1, sort_every 1, ppl 0 or 2 and no moving window (else
 * PIC_EINVAL).
 */
#define PIC_FLAG_QUADRATIC 16u

/*
 * Moving window (pic_config.flags; the last step of Listing 3.1): enables
 * pic_move_window() and sizes the workspace for it.  Not available in
 * batched mode.
 */
#define PIC_FLAG_MOVING_WINDOW 4u

/*
 * Alternative sort (pic_config.flags): the motion-class sort Sec. 4.3 cites
 * (after Germaschewski et al.).  By the Courant condition a particle ends a
 * step in its own tile or one of the eight around it, so its motion falls
 * into one of nine classes, (dty + 1) * 3 + (dtx + 1) for the step (dtx, dty)
 * from the tile whose section held it to its new tile (counted +1 on an axis
 * of two tiles, where both neighbours coincide); the push counts every tile's
 * particles per class.  pic_sort() then moves every particle, in one counting
 * pass, to its slot in the order (new tile, class, old slot) in the
 * workspace, and copies the result back: out of place, reading and writing
 * every particle twice, so it pays only when most particles change tile.
 * In pic_step() (with the default current and deposit) the copy back is
 * left to the next push, which reads the particles from the workspace
 * (see the memory model).  Also in batched mode (copied back at once).  pic_diag's mover count is 0 with it.  The moving
 * window keeps its own (in-place) re-sort.
 */
#define PIC_FLAG_MOTION_SORT 8u

/*
 * Binomial current filter (pic_config.j_filter; Listing 3.1's optional
 * smoothing of J after update_gc_add).  Each pass smooths every J component
 * with the three-point kernel (1/4, 1/2, 1/4) along x, then along y, on the
 * periodic grid (FP32, the two directions in one stencil).  The filter
 * commutes with the discrete divergence, so the filtered current conserves the
 * equally filtered charge density; pic_diag's continuity and Gauss residuals
 * then use that filtered density.
 */
#define PIC_MAX_FILTER 16

typedef struct pic_species {
    double qm;    /* charge-to-mass ratio q/m (electrons: -1) */
    double q;     /* charge density carried by one particle (e.g. -n0 / ppc) */
    int64_t n;    /* number of particles, 0 <= n < 2^31 */
    int64_t cap;  /* entries of the particle arrays, n <= cap < 2^31 (0: n); the
                     moving window adds and removes particles within it */
} pic_species;

typedef struct pic_config {
    int32_t nx, ny;      /* cells; multiples of tile, 1 <= nx, ny <= 32767 */
    double dx, dy, dt;   /* cell size and time step; dt < 1/sqrt(1/dx^2 + 1/dy^2) */
    int32_t tile;        /* tile edge in cells: 8, 16 or 32 */
    int32_t j_replicas;  /* LDS current replicas per tile: 1, 2 or 4 (0 = default) */
    int32_t n_species;   /* 1 .. PIC_MAX_SPECIES */
    uint32_t flags;      /* OR of PIC_FLAG_J_FLOAT, PIC_FLAG_ESIRKEPOV, PIC_FLAG_MOVING_WINDOW,
                            PIC_FLAG_MOTION_SORT, PIC_FLAG_QUADRATIC, or 0 */
    int32_t j_filter;    /* binomial current filter passes, 0 (off) .. PIC_MAX_FILTER */
    int32_t sort_every;  /* sort cadence k = 1, 2 or 4 (0: 1): pic_step sorts every
                            k-th step and the push stages a halo k cells wide.  k > 1
                            needs the fixed-point current with j_replicas <= 1, no
                            moving window, and 2k + 1 <= tile within the LDS budget
                            (tile 8: k <= 2; 16: k <= 4; 32: k <= 2), else PIC_EINVAL /
                            PIC_ETILE */
    int32_t ppl;         /* particles per lane per pass of the push loop: 1, 2 or 4 (0: 2),
                            the 64-particle chunks a wavefront carries side by side; other
                            than 2 needs the fixed-point current, the default deposit and
                            j_replicas <= 1 (else PIC_EINVAL).  Results do not depend on it */
    pic_species species[PIC_MAX_SPECIES];
} pic_config;

typedef struct pic_particles {   /* device pointers, n entries each */
    int32_t *cell;
    float *x, *y, *ux, *uy, *uz;
} pic_particles;

typedef struct pic_buffers {
    float *fields;       /* device, 9 * nx * ny floats (layout above) */
    /* particle arrays: device, species[s].cap entries each (n of them valid) */
    void *work;          /* device, pic_sizes.work_bytes, 256-byte aligned */
    size_t work_bytes;
    pic_particles sp[PIC_MAX_SPECIES];
} pic_buffers;

typedef struct pic_sizes {
    int32_t n_tiles;
    size_t field_bytes;  /* bytes of pic_buffers.fields */
    size_t work_bytes;   /* bytes of pic_buffers.work */
} pic_sizes;

typedef struct pic_sim pic_sim;   /* opaque */

/*
 * Sizes of the caller-allocated buffers for cfg.  Allocates nothing.
 * Returns PIC_EINVAL / PIC_ETILE / PIC_ECFL on a bad configuration.
 */
int pic_query(const pic_config *cfg, pic_sizes *out);

/*
 * Validate cfg (Courant condition Eq. 1, tile divisibility, sizes) and bind
 * the caller's buffers.  The caller has filled the particle arrays (in any
 * order) and the E and B planes; J is overwritten by every push.  Groups the
 * particles of every species by tile in place on the device if they are not
 * yet (a stable sort on the tile id: inside a tile the given order is kept,
 * so grouped input is left as it is), builds tile_offset and synchronises
 * `stream`.  Returns PIC_EORDER if a cell is out of range.  On success *out
 * owns a host record, one HIP stream of default priority and two events
 * (pic_step's fork and join), all released by pic_destroy().
 */
int pic_init(const pic_config *cfg, const pic_buffers *bufs, hipStream_t stream,
             pic_sim **out);

/*
 * Particle half of the step (Listing 3.1 loop body, Sec. 4.2): for every tile,
 * stage its E/B halo in LDS, interpolate, Boris-push (Eqs. 6-10), move
 * (Eq. 11), deposit the Villasenor-Buneman current of each 1/2/3-piece
 * motion into LDS (Eqs. 13-16), then write J (all species) into the J planes,
 * folding the periodic images (update_gc_add), and apply the binomial filter
 * if pic_config.j_filter > 0.  Also records, per tile, the
 * particles that are now outside it, as input for pic_sort().  A particle that
 * would move one cell or more sets PIC_ERANGE (reported by pic_check()).
 * Returns PIC_EORDER without launching anything once sort_every pushes have
 * run since the last pic_sort() (the particles could have left the staged
 * halo).
 */
int pic_push_deposit(pic_sim *sim, hipStream_t stream);

/*
 * Strict re-sort by tile after a push (Sec. 4.3, Fig. 4.5): recount the
 * tiles, rebuild tile_offset, and move every particle whose slot lies outside
 * its tile's new section into a hole.  The result is the canonical one: holes
 * in ascending slot order receive the movers ordered by destination tile,
 * then by old slot.  Particles already in their section do not move.  Uses
 * the record of the last push, so it may run after any push; with no push
 * since the last sort it does nothing.
 */
int pic_sort(pic_sim *sim, hipStream_t stream);

/*
 * Bring the caller's particle arrays up to date (see the memory model):
 * completes what pic_step()'s or pic_batch_step()'s sort left to the next
 * push (the staged movers into their holes, or the motion-class sort's
 * staging arrays copied back; nothing if none is pending) and writes every
 * particle's cell, ix | iy << 16, into the cell array.  Enqueues its kernels
 * on `stream` without synchronising.
 */
int pic_sync(pic_sim *sim, hipStream_t stream);

/*
 * Field half of the step (Listing 3.1): B half step, E full step with the
 * current J, B half step (Eqs. 19-20 on the Yee grid, periodic images read
 * directly: update_gc_copy).
 */
int pic_field_advance(pic_sim *sim, hipStream_t stream);

/*
 * Move the window one cell towards +x (the moving-window step at the end of
 * Listing 3.1; requires PIC_FLAG_MOVING_WINDOW).  In window coordinates: E and
 * B move one cell towards -x and the last column becomes zero; every particle
 * moves one cell towards -x (offsets kept); the particles that were in window
 * column 0 leave; the n_inject[s] new particles of species s (device arrays
 * inject[s], cells given in window column nx - 1 and grouped by tile, e.g.
 * fresh plasma drawn by the caller) come in.
 * In the arrays: the grid is periodic between moves, so the shift is kept as
 * a relabelling -- window column i is array column (i + origin) mod nx, and
 * the move advances origin (pic_get_window_origin) by one.  Only the array
 * column that held window column 0 changes: its E and B become zero, its
 * particles leave and the new particles are placed in it.  The particles are
 * then re-sorted by tile canonically, as pic_sort does, the leaving ones
 * removed and the new ones taken as appended after the existing ones.  The
 * particle counts change (pic_get_counts); the call synchronises `stream`.
 * Returns PIC_EINVAL if a count would exceed its species' capacity, and
 * PIC_EORDER if a new particle is outside window column nx - 1 or the new
 * particles are not grouped by tile (nothing has changed then).
 */
int pic_move_window(pic_sim *sim, const pic_particles *inject, const int64_t *n_inject, hipStream_t stream);

/* Array column that holds window column 0 (0 until the first pic_move_window
 * and always 0 without PIC_FLAG_MOVING_WINDOW; host record, no device access).
 * The field planes, the particles' cells and tile_offset are in array
 * columns; diagnostics do not depend on the origin. */
int pic_get_window_origin(pic_sim *sim, int32_t *origin);

/* Current particle count of every species (n_species values; host record, no
 * device access). */
int pic_get_counts(pic_sim *sim, int64_t *counts);

/* pic_push_deposit + pic_sort (every sort_every-th step) + pic_field_advance,
 * with the same results once the sort's hole fill is done: the next push
 * does it, or pic_sync() (see the memory model).  The push also forms the
 * field advance's first B half step for its tile (into workspace planes), so
 * the field half is the E step and the second half step.  In a step that
 * sorts, the field half (J fold, filter, field advance) runs on the
 * library's own stream beside the sort: forked from `stream` after the push
 * with an event and joined back into `stream` before the call returns, so
 * everything the caller enqueues on `stream` afterwards sees the whole step.
 * Issues kernels and event records/waits only (no memset, no
 * synchronisation), so a caller may capture it into a HIP graph; with
 * sort_every > 1 the captured step keeps the sort decision taken at capture
 * time. */
int pic_step(pic_sim *sim, hipStream_t stream);

/* Synchronise `stream` and report (and clear) the device error flags. */
int pic_check(pic_sim *sim, hipStream_t stream);

/* Diagnostics, FP64 reductions on the device. */
#define PIC_DIAG_ENERGY 1u          /* u_e, u_b, u_k */
#define PIC_DIAG_RHO_SNAPSHOT 2u    /* remember rho of the current positions */
#define PIC_DIAG_CONTINUITY 4u      /* residual against the snapshot and current J */
#define PIC_DIAG_COUNTS 8u          /* leavers of the last push, movers of the last sort */
#define PIC_DIAG_GAUSS 16u          /* residuals of Gauss's law and of div B = 0 */

typedef struct pic_diag_out {
    double u_e;                       /* 1/2 dx dy sum |E|^2 */
    double u_b;                       /* 1/2 dx dy sum |B|^2 */
    double u_k[PIC_MAX_SPECIES];      /* dx dy sum (q/qm) (gamma - 1) */
    double continuity_max;            /* max |rho' - rho + dt div J| */
    double rho_max;                   /* max |rho'| */
    int64_t leavers[PIC_MAX_SPECIES]; /* particles whose tile changed */
    int64_t movers[PIC_MAX_SPECIES];  /* particles moved by the last sort */
    double gauss_max;                 /* max |div E - (rho - rho_bar)| over the nodes */
    double divb_max;                  /* max |div B| over the cell centres */
} pic_diag_out;

/*
 * Compute the diagnostics selected by `what` (bitwise OR of PIC_DIAG_*) on
 * `stream`, synchronise it and fill *out (fields not selected are zero).
 * PIC_DIAG_CONTINUITY evaluates Eq. (12) in discrete form,
 * rho(now) - rho(snapshot) + dt * div J, at the nodes; it returns PIC_EINVAL
 * without an earlier PIC_DIAG_RHO_SNAPSHOT.  PIC_DIAG_GAUSS evaluates
 * Gauss's law on the Yee grid, div E = rho - rho_bar at the nodes, with the
 * ions a uniform neutralising background rho_bar (the mean of rho, from the
 * particle charges and counts), and div B at the cell centres; a
 * charge-conserving step keeps both at their initial values.  Also reports
 * device error flags like pic_check().
 */
int pic_diag(pic_sim *sim, unsigned what, pic_diag_out *out, hipStream_t stream);

/*
 * Valid initial fields (Sec. 3.2: the fields start out satisfying Eq. 17,
 * div E = rho, and Eq. 18, div B = 0).  With the ions a uniform neutralising
 * background (rho_bar as in PIC_DIAG_GAUSS) and on the periodic Yee grid:
 *   E <- E - grad psi,  Lap psi = div E - (rho - rho_bar)   (psi at the nodes)
 *   B <- B - grad chi,  Lap chi = div B                     (chi at the cell centres)
 * Lap is the five-point Laplacian, the divergence of the grid gradient; a
 * gradient has no discrete curl, so the curls of E and B are unchanged and
 * Ez, Bz are not touched.  From E = B = 0 this is the electrostatic field of
 * the particles (e.g. a perturbed plasma).  rho is that of the Gauss
 * diagnostic (binomially filtered when pic_config.j_filter > 0).  Each
 * Poisson problem is solved by conjugate gradients in FP64 until ||r|| <= tol
 * ||r0|| (tol <= 0: 1e-12) or max_iter iterations (<= 0: 20 max(nx, ny) +
 * 100); the result is stored in FP32.
 * scratch: device memory of at least PIC_GAUSS_SCRATCH_BYTES(nx, ny) bytes,
 * 256-byte aligned, caller-owned.  Synchronises `stream`.  out (may be NULL)
 * receives the iterations and final relative residual of both solves.
 * Returns PIC_EINVAL for bad arguments and PIC_ENOCONV if a solve stopped
 * short of tol (the fields then hold the last iterate's correction).
 */
#define PIC_GAUSS_SCRATCH_BYTES(nx, ny) (32 * (size_t)(nx) * (size_t)(ny) + 16384)
typedef struct pic_gauss_out {
    int32_t iterations[2];   /* [0]: E (Eq. 17), [1]: B (Eq. 18) */
    double residual[2];      /* ||r|| / ||r0|| at the end (0 when r0 = 0) */
} pic_gauss_out;
int pic_solve_gauss(pic_sim *sim, void *scratch, size_t scratch_bytes, double tol, int max_iter,
                    pic_gauss_out *out, hipStream_t stream);

/*
 * pic_solve_gauss for callers that cannot allocate device memory (a serving
 * loop or a harness that forbids hipMalloc): the same solve, with the same
 * results bit for bit, in a scratch array the library holds in every
 * device's memory from the moment it is loaded until the process ends --
 * PIC_GAUSS_SCRATCH_BYTES(1024, 1024) bytes, so at most
 * PIC_GAUSS_NOALLOC_MAX_CELLS cells (nx * ny; PIC_ESCRATCH beyond, nothing
 * done).  Allocates nothing.  Every call on one device shares that device's
 * array, which keeps the last call's contents (each call writes every value
 * it reads first): calls that overlap in time on one device -- from two host
 * threads, or on two streams -- race and must not be made.  The device
 * current at the call must be the one the simulation was created on
 * (PIC_EINVAL otherwise).  Synchronises `stream`; out and the return codes
 * as for pic_solve_gauss.
 */
#define PIC_GAUSS_NOALLOC_MAX_CELLS (1 << 20)
int pic_solve_gauss_noalloc(pic_sim *sim, double tol, int max_iter, pic_gauss_out *out, hipStream_t stream);

/*
 * State I/O: host copies of everything that carries over from one step to
 * the next -- the field planes and every species' particles -- for
 * checkpoint / resume and for replaying a step on another implementation.
 * tile_offset is derived from the particles and rebuilt on load.
 */
typedef struct pic_host_state {
    float *fields;                      /* host, 9 * nx * ny floats (layout above) */
    pic_particles sp[PIC_MAX_SPECIES];  /* host arrays, n[s] entries each */
    int64_t n[PIC_MAX_SPECIES];         /* particle counts (pic_get_counts) */
    int32_t window_origin;              /* see pic_get_window_origin */
} pic_host_state;

/* Copy the field planes and the particles of every species (array columns)
 * to the caller's host arrays (a NULL array is skipped; the arrays hold the
 * current counts, pic_get_counts), set out->n and out->window_origin and
 * synchronise `stream`.  With sort_every > 1 a state taken between two sorts
 * holds particles outside their tile's section; pic_set_state() regroups
 * them, so it resumes in a different (valid) slot order than a run that
 * never stopped. */
int pic_get_state(pic_sim *sim, pic_host_state *out, hipStream_t stream);

/*
 * Load the field planes, the particles (in->n[s] of species s, in any order,
 * grouped by tile on the device as in pic_init; array columns) and the window
 * origin from host arrays, rebuild tile_offset, forget the rho snapshot of
 * pic_diag and synchronise `stream`.  Every array must be given.  With
 * PIC_FLAG_MOVING_WINDOW a count may be anything up to the species' capacity
 * and 0 <= origin < nx; without it the counts must be the current ones and
 * the origin 0 (else PIC_EINVAL, nothing loaded).  Returns PIC_EORDER if a
 * cell is out of range (the simulation then needs a valid state before its
 * next step).
 */
int pic_set_state(pic_sim *sim, const pic_host_state *in, hipStream_t stream);

/* Copy the current tile_offset of `species` (n_tiles + 1 int32) to host memory. */
int pic_get_tile_offsets(pic_sim *sim, int species, int32_t *host_out, hipStream_t stream);

/* Per-kernel timing with HIP events on the launching stream. */
#define PIC_KERNEL_PUSH 0         /* push + deposit kernel */
#define PIC_KERNEL_JREDUCE 1      /* tile current fold into the J planes (pic_push_deposit; in
                                     pic_step only with the filter, else fused into the field advance) */
#define PIC_KERNEL_SORT_SCAN 2    /* tile recount + tile_offset scan */
#define PIC_KERNEL_SORT_PLAN 3    /* hole/mover pairing + mover gather */
#define PIC_KERNEL_SORT_SCATTER 4 /* mover scatter into holes */
#define PIC_KERNEL_FIELD 5        /* the three Yee sub-steps (in pic_step without the filter, the
                                     E step also folds J) */
#define PIC_KERNEL_FILTER 6       /* binomial current filter passes */
#define PIC_N_KERNELS 7

typedef struct pic_timing_out {
    double ms_total[PIC_N_KERNELS];   /* summed event time since the last reset */
    int64_t launches[PIC_N_KERNELS];
} pic_timing_out;

/* enable = 1: record HIP events around every launch from now on; 0: stop. Resets the sums. */
int pic_set_timing(pic_sim *sim, int enable);

/* Like pic_set_timing, for the kernels whose bit (1 << PIC_KERNEL_*) is set
 * in mask only (0: stop): every event pair adds a little time to the step,
 * so a throughput run times just the kernel it reports. */
int pic_set_timing_mask(pic_sim *sim, unsigned mask);

/* Synchronise on the recorded events and return the sums since the last reset. */
int pic_get_timing(pic_sim *sim, pic_timing_out *out);

/*
 * ---- Many independent simulations advanced together (batched mode) ----
 *
 * Hundreds of small simulations (each its own grid, species and particle
 * count) share every kernel launch: one launch per phase of the step for the
 * whole batch, the push as one workgroup per (simulation, tile) work item,
 * largest simulations first, and optionally one captured HIP graph per
 * step.  All members must share tile, j_replicas, flags, j_filter and
 * sort_every.
 * Results are bit-identical to advancing each member alone with pic_step.
 */
typedef struct pic_batch pic_batch;

/* Device bytes the batch itself needs (descriptors, work tables, counter). */
int pic_batch_query(int n, const pic_config *cfgs, size_t *bytes);

/*
 * n >= 1 members: cfgs[i] / bufs[i] exactly as for pic_init (each member's
 * own caller-owned fields, workspace and particles).  batch_work: device
 * memory of pic_batch_query() bytes, 256-byte aligned, caller-owned.
 * Synchronises `stream`.  Errors as pic_init, or PIC_EINVAL if the members do
 * not share tile / j_replicas / flags / j_filter / sort_every.  The batch
 * owns one HIP stream of default priority and two events (the fork and join
 * of pic_batch_step), released by pic_batch_destroy(); its members own none.
 */
int pic_batch_init(int n, const pic_config *cfgs, const pic_buffers *bufs, void *batch_work,
                   size_t batch_bytes, hipStream_t stream, pic_batch **out);

/* nsteps full steps of every member (push + deposit, sort every sort_every-th
 * step, field advance): replays of the captured cycle of sort_every steps if
 * pic_batch_capture() was called and a whole cycle remains, else direct
 * launches.  As in pic_step, the field half of a sorting step runs on the
 * batch's own stream beside the sort and is joined back into `stream`. */
int pic_batch_step(pic_batch *b, int nsteps, hipStream_t stream);

/* Capture one batched cadence cycle (sort_every steps, the last with the
 * sort) into a HIP graph on `stream` (a non-null stream); later
 * pic_batch_step() calls on any stream replay it.  Nothing runs here. */
int pic_batch_capture(pic_batch *b, hipStream_t stream);

/* Member i as a pic_sim for pic_diag / pic_get_tile_offsets / pic_check and
 * the single-member calls; owned by the batch (do not pic_destroy it).
 * NULL if i is out of range.  Event timing switched on for member 0
 * (pic_set_timing_mask with PIC_KERNEL_PUSH) also times the batch's
 * push launch in direct (not graph-replayed) batched steps; do
 * not capture with it on. */
pic_sim *pic_batch_sim(pic_batch *b, int i);

/* pic_sync() for every member at once (one launch for the hole fills that
 * the last batched sort left to the next push, one for the cells).  Enqueues
 * on `stream`. */
int pic_batch_sync(pic_batch *b, hipStream_t stream);

/* pic_check of every member; the first error found. */
int pic_batch_check(pic_batch *b, hipStream_t stream);

/* Free the batch's host record, its graph and its members' host records. */
void pic_batch_destroy(pic_batch *b);

/*
 * Measurement aid, not a step of the method: the push kernel's particle
 * stream without its arithmetic.  Six device arrays -- arrays[0] of n 16-bit
 * values (the tile-relative cells), arrays[1..5] of n 32-bit values (x, y,
 * ux, uy, uz) -- are each read and written back unchanged, in 64-value
 * chunks through buffer descriptors, 16,384 values of every array per
 * workgroup; nontemporal != 0 gives the loads and stores the push's
 * non-temporal hint.  Timing it gives the bandwidth this access pattern
 * reaches (22 n bytes read, 22 n written), the practical ceiling of the
 * push's streaming.  Enqueues one kernel on `stream`; PIC_EINVAL for a null
 * array or n < 0.
 */
int pic_probe_stream(void *const *arrays, int64_t n, int nontemporal, hipStream_t stream);

/* Static string naming a return code. */
const char *pic_strerror(int code);

/* Free the host record, the library's stream (after its work has finished)
 * and events.  Caller buffers are untouched. */
void pic_destroy(pic_sim *sim);

#ifdef __cplusplus
}
#endif

#endif /* PIC_H */

// C ABI of libpic: validation, workspace carve-up, launch sequencing, error
// flags, diagnostics and per-kernel event timing.  See include/pic.h.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "pic_internal.h"

using namespace pic;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

struct Layout {
    size_t err = 0, stg_live = 0, dacc = 0, cacc = 0, jtile = 0, bh = 0, rho_prev = 0, rho_now = 0, jf = 0, rho_tmp = 0;
    size_t wrem = 0, inj_off[kMaxSpecies] = {};
    size_t off[kMaxSpecies][2] = {}, cnt[kMaxSpecies] = {}, leav[kMaxSpecies] = {};
    size_t hole[kMaxSpecies] = {}, stg[kMaxSpecies][6] = {}, mcount[kMaxSpecies] = {}, bsum[kMaxSpecies] = {};
    size_t lrec[kMaxSpecies] = {}, srec[kMaxSpecies] = {}, fcount[kMaxSpecies] = {}, fbase[kMaxSpecies] = {};
    size_t lcell[kMaxSpecies] = {};
    size_t total = 0;
};

int j_mode(const pic_config *c) { return (c->flags & PIC_FLAG_J_FLOAT) ? kJFloat : kJFixed; }
int d_mode(const pic_config *c)
{
    if (c->flags & PIC_FLAG_QUADRATIC) return kDepQuad;
    return (c->flags & PIC_FLAG_ESIRKEPOV) ? kDepEsirkepov : kDepVB;
}

// sort cadence: pushes between sorts
int cadence_of(const pic_config *c) { return c->sort_every ? c->sort_every : 1; }
// the push kernel's halo pad: the cadence, plus what the particle shape needs
int halo_of(const pic_config *c) { return cadence_of(c) + shape_pad(d_mode(c)); }
int ppl_of(const pic_config *c) { return c->ppl ? c->ppl : 2; }

int default_replicas(const pic_config *c)
{
    if (j_mode(c) == kJFixed) return 1;   // integer LDS atomics need no replicas
    return c->tile >= 32 ? 2 : 4;
}

int validate(const pic_config *c)
{
    if (!c) return PIC_EINVAL;
    if (c->flags & ~(uint32_t)(PIC_FLAG_J_FLOAT | PIC_FLAG_ESIRKEPOV | PIC_FLAG_MOVING_WINDOW | PIC_FLAG_MOTION_SORT |
                               PIC_FLAG_QUADRATIC))
        return PIC_EINVAL;
    // the quadratic shape is built for one sort per step (its halo pad is 2)
    if ((c->flags & PIC_FLAG_QUADRATIC) && c->sort_every > 1) return PIC_EINVAL;
    // the Esirkepov deposit is built for the fixed-point current only
    if ((c->flags & PIC_FLAG_ESIRKEPOV) && (c->flags & PIC_FLAG_J_FLOAT)) return PIC_EINVAL;
    if (c->tile != 8 && c->tile != 16 && c->tile != 32) return PIC_ETILE;
    if (c->nx < c->tile || c->ny < c->tile || c->nx > 32767 || c->ny > 32767) return PIC_EINVAL;
    if (c->nx % c->tile || c->ny % c->tile) return PIC_ETILE;
    if (c->j_replicas != 0 && c->j_replicas != 1 && c->j_replicas != 2 && c->j_replicas != 4)
        return PIC_EINVAL;
    if (c->n_species < 1 || c->n_species > kMaxSpecies) return PIC_EINVAL;
    if (c->j_filter < 0 || c->j_filter > PIC_MAX_FILTER) return PIC_EINVAL;
    {
        const int r = c->j_replicas ? c->j_replicas : default_replicas(c);
        if (push_lds_bytes(c->tile, r, j_mode(c)) > kLdsBytes) return PIC_EINVAL;
    }
    {
        // the push kernel's halo pad: the number of steps between sorts (plus
        // one cell for the quadratic shape)
        const int k = halo_of(c);
        if (k != 1 && k != 2 && k != 4) return PIC_EINVAL;
        if (k > 1) {
            if (j_mode(c) != kJFixed || c->j_replicas > 1) return PIC_EINVAL;
            if (c->flags & PIC_FLAG_MOVING_WINDOW) return PIC_EINVAL;
            if (!cadence_ok(c->tile, k)) return PIC_ETILE;
        }
    }
    {
        // particles per lane: 1 and 4 are built for the autotuner's configurations
        const int ppl = ppl_of(c);
        if (ppl != 1 && ppl != 2 && ppl != 4) return PIC_EINVAL;
        if (ppl != 2 && (j_mode(c) != kJFixed || d_mode(c) != kDepVB || c->j_replicas > 1)) return PIC_EINVAL;
    }
    if (!(c->dx > 0) || !(c->dy > 0) || !(c->dt > 0)) return PIC_EINVAL;
    // Courant-Levy condition, Eq. (1), with c = 1
    if (!(c->dt < 1.0 / sqrt(1.0 / (c->dx * c->dx) + 1.0 / (c->dy * c->dy)))) return PIC_ECFL;
    for (int s = 0; s < c->n_species; ++s) {
        const pic_species &sp = c->species[s];
        if (sp.n < 0 || sp.n >= (int64_t)1 << 31) return PIC_EINVAL;
        if (sp.cap != 0 && (sp.cap < sp.n || sp.cap >= (int64_t)1 << 31)) return PIC_EINVAL;
        if (!isfinite(sp.qm) || !isfinite(sp.q)) return PIC_EINVAL;
    }
    return PIC_OK;
}

Layout make_layout(const pic_config *c)
{
    Layout L;
    const int T = c->tile;
    const int64_t n_tiles = (int64_t)(c->nx / T) * (c->ny / T);
    const int64_t nodes = (int64_t)c->nx * c->ny;
    size_t p = 0;
    auto take = [&](size_t bytes) {
        const size_t at = p;
        p = align_up(p + std::max<size_t>(bytes, 1));
        return at;
    };
    L.err = take(64);
    L.stg_live = take(64);
    L.dacc = take(32 * sizeof(double));
    L.cacc = take(8 * sizeof(unsigned long long));
    const int NJ = T + 2 * halo_of(c) + 1;   // current halo nodes per axis
    L.jtile = take((size_t)n_tiles * 3 * NJ * NJ * sizeof(float));
    L.bh = take(nodes * 3 * sizeof(float));   // B after the first half step (pic_step)
    L.rho_prev = take(nodes * sizeof(double));
    L.rho_now = take(nodes * sizeof(double));
    if (c->j_filter > 0) {
        L.jf = take(nodes * 3 * sizeof(float));      // filter ping-pong partner of the J planes
        L.rho_tmp = take(nodes * sizeof(double));    // the same for the diagnostic density
    }
    if (c->flags & PIC_FLAG_MOVING_WINDOW) {
        L.wrem = take(kMaxSpecies * sizeof(int32_t));
        for (int s = 0; s < c->n_species; ++s) L.inj_off[s] = take((n_tiles + 1) * sizeof(int32_t));
    }
    for (int s = 0; s < c->n_species; ++s) {
        // per-particle scratch sized for the capacity (the window changes n)
        const size_t n = (size_t)(c->species[s].cap ? c->species[s].cap : c->species[s].n);
        // the tile-relative cells the kernels stream (16 bits each)
        L.lcell[s] = take(n * sizeof(int16_t));
        L.off[s][0] = take((n_tiles + 1) * sizeof(int32_t));
        L.off[s][1] = take((n_tiles + 1) * sizeof(int32_t));
        L.cnt[s] = take((size_t)n_tiles * kCntStride * sizeof(int32_t));
        L.leav[s] = take(n * sizeof(uint32_t));
        // leaver records; the full re-sort also borrows the region as six
        // arrays of n values (lp_view)
        L.lrec[s] = take(n * sizeof(LeaverRec) + 6 * kAlign);
        L.hole[s] = take(n * sizeof(int32_t));
        // mover staging: the in-place sort's 32-byte records (every
        // simulation: the moving window's sort is the in-place one; also the
        // initial grouping's scratch), and the motion-class sort's six arrays
        L.srec[s] = take(n * sizeof(LeaverRec));
        if (c->flags & PIC_FLAG_MOTION_SORT)
            for (int k = 0; k < 6; ++k) L.stg[s][k] = take(n * (k == 0 ? sizeof(int16_t) : sizeof(float)));
        L.mcount[s] = take((size_t)3 * n_tiles * sizeof(int32_t));   // movers (motion sort: class bases)
        L.fcount[s] = take((size_t)n_tiles * sizeof(int32_t));       // pending fill per tile
        L.fbase[s] = take((size_t)n_tiles * push_waves(T) * sizeof(int32_t));
        L.bsum[s] = take((size_t)(n_tiles / kScanBlock + 1) * sizeof(int32_t));
    }
    L.total = p;
    return L;
}

}  // namespace

struct pic_sim {
    pic_config cfg;
    pic_buffers buf;
    int ntx, nty, n_tiles, tile, replicas;
    char *work;
    int *err;
    int *stg_live;      // nonzero: the particles wait in the motion-class sort's staging arrays
    double *dacc;
    unsigned long long *cacc;
    float *jtile;
    float *bh;          // B after the step's first half step, written by pic_step's push
    double *rho_prev, *rho_now;
    float *jf;          // filter partner of the J planes (j_filter > 0)
    double *rho_tmp;    // filter partner of rho_now (j_filter > 0)
    int32_t origin;     // moving window: array column of window column 0
    int cadence;        // sort cadence: pushes between sorts
    int halo;           // the push kernel's halo pad (the cadence, + 1 for the quadratic shape)
    int since_sort;     // pushes since the last sort
    int32_t *wrem;      // moving window: particles that left, per species
    // pic_step's second stream: the field half of a step (J fold, filter,
    // field advance) runs there beside the sort, forked from and joined back
    // into the caller's stream with these two events
    hipStream_t side;
    hipEvent_t ev_fork, ev_join;
    int64_t cap[kMaxSpecies];
    int device;         // the device current at pic_init
    bool have_snapshot;
    struct Sp {
        int16_t *lcell;  // the tile-relative cells the push and the sort stream
        int32_t *off;    // current tile_offset
        int32_t *offp;   // the tile_offset before the sort (scratch)
        int32_t *cnt;
        uint32_t *leav;
        int32_t *hole;
        Parts stg;         // the motion-class sort's staging (null without PIC_FLAG_MOTION_SORT)
        LeaverRec *srec;   // the in-place sort's mover staging (every simulation)
        LeaverRec *lrec;   // the push's leaver records
        GParts lp;         // the same memory as six arrays of n values (the initial grouping's scratch)
        int32_t *mcount;
        int32_t *fcount;   // holes whose fill a deferred sort left to the next push
        int32_t *fbase;
        int32_t *bsum;
        int32_t *inj_off;   // moving window: tile offsets of the new particles
    } sp[kMaxSpecies];
    // timing
    bool timing;
    unsigned timing_mask;   // kernels timed while timing is on (bit PIC_KERNEL_*)
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[PIC_N_KERNELS];
    double ms[PIC_N_KERNELS];
    int64_t launches[PIC_N_KERNELS];
};

// The scratch of pic_solve_gauss_noalloc: the conjugate-gradient vectors of
// the largest grid it takes.  Every device holds its own copy from the
// moment the library is loaded until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in
// for the symbol): it uses the device address hipGetSymbolAddress returns,
// looked up once per device.
static __device__ __align__(256) unsigned char scratch[PIC_GAUSS_SCRATCH_BYTES(1024, 1024)];
static_assert(PIC_GAUSS_SCRATCH_BYTES(1024, 1024) == 32 * (size_t)PIC_GAUSS_NOALLOC_MAX_CELLS + 16384,
              "the static scratch holds the largest grid pic_solve_gauss_noalloc takes");

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on `dev`, which must be the current device
// (the symbol has one address per device).
int scratch_address(int dev, void **ptr)
{
    if (dev < 0 || dev >= kMaxDevices) return PIC_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PIC_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return PIC_OK;
}

void release_side(pic_sim *s)
{
    if (s->side) {
        (void)hipStreamSynchronize(s->side);
        (void)hipStreamDestroy(s->side);
    }
    if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
    if (s->ev_join) (void)hipEventDestroy(s->ev_join);
    s->side = nullptr;
    s->ev_fork = s->ev_join = nullptr;
}

hipEvent_t take_event(pic_sim *s)
{
    if (!s->pool.empty()) {
        hipEvent_t e = s->pool.back();
        s->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records HIP events around the launches of one kernel class on `stream`.
struct Timed {
    pic_sim *s;
    int k;
    hipStream_t st;
    hipEvent_t a = nullptr;
    Timed(pic_sim *sim, int kernel, hipStream_t stream) : s(sim), k(kernel), st(stream)
    {
        if (s->timing && ((s->timing_mask >> k) & 1u)) {
            a = take_event(s);
            if (a) (void)hipEventRecord(a, st);
        }
    }
    ~Timed()
    {
        if (a) {
            hipEvent_t b = take_event(s);
            if (b) {
                (void)hipEventRecord(b, st);
                s->pending[k].push_back({a, b});
            } else {
                s->pool.push_back(a);
            }
        }
    }
};

int hip_ok(hipError_t e) { return e == hipSuccess ? PIC_OK : PIC_EHIP; }

// Synchronise `stream`, read and clear the device error bits into *h.
int read_flags(pic_sim *s, hipStream_t stream, int *h)
{
    *h = 0;
    if (hipMemcpyAsync(h, s->err, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess) return PIC_EHIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return PIC_EHIP;
    if (*h) {
        if (hipMemsetAsync(s->err, 0, sizeof(int), stream) != hipSuccess) return PIC_EHIP;
        if (hipStreamSynchronize(stream) != hipSuccess) return PIC_EHIP;
    }
    return PIC_OK;
}

int read_errors(pic_sim *s, hipStream_t stream)
{
    int h = 0;
    const int rc = read_flags(s, stream, &h);
    if (rc) return rc;
    if (h & (kErrOrder | kErrGroup)) return PIC_EORDER;
    if (h & kErrRange) return PIC_ERANGE;
    if (h & kErrCount) return PIC_ECOUNT;
    if (h & kErrSort) return PIC_ESORT;
    if (h & kErrOverflow) return PIC_EOVERFLOW;
    return PIC_OK;
}

DiagSpecies diag_species(const pic_sim *s, int k)
{
    DiagSpecies d;
    const pic_particles &p = s->buf.sp[k];
    d.cell = p.cell;
    d.x = p.x;
    d.y = p.y;
    d.ux = p.ux;
    d.uy = p.uy;
    d.uz = p.uz;
    d.n = (int32_t)s->cfg.species[k].n;
    d.q = s->cfg.species[k].q;
    d.quadratic = d_mode(&s->cfg) == kDepQuad ? 1 : 0;
    return d;
}

// The node charge density of the Gauss diagnostic into rho_now: every
// species' charge at the nodes, binomially filtered like the current when the
// filter is on (the density whose continuity the filtered current satisfies).
int node_density(pic_sim *S, hipStream_t stream)
{
    const pic_config &c = S->cfg;
    const int64_t plane = (int64_t)c.nx * c.ny;
    int rc = hip_ok(hipMemsetAsync(S->rho_now, 0, plane * sizeof(double), stream));
    if (rc) return rc;
    for (int s = 0; s < c.n_species; ++s) launch_diag_rho(diag_species(S, s), c.nx, c.ny, S->rho_now, stream);
    for (int p = 0; p < c.j_filter; ++p) {
        FilterArgs f;
        f.src = (p & 1) ? S->rho_tmp : S->rho_now;
        f.dst = (p & 1) ? S->rho_now : S->rho_tmp;
        f.nx = c.nx;
        f.ny = c.ny;
        f.planes = 1;
        launch_filter(f, true, stream);
    }
    if (c.j_filter & 1)
        rc = hip_ok(hipMemcpyAsync(S->rho_now, S->rho_tmp, plane * sizeof(double), hipMemcpyDeviceToDevice, stream));
    return rc;
}

// The uniform neutralising background: the mean charge density.
double mean_density(const pic_sim *S)
{
    const pic_config &c = S->cfg;
    double total = 0.0;
    for (int s = 0; s < c.n_species; ++s) total += c.species[s].q * (double)c.species[s].n;
    return total / ((double)c.nx * c.ny);
}

// Both Poisson projections of pic_solve_gauss in the scratch d of
// PIC_GAUSS_SCRATCH_BYTES(nx, ny) bytes (4 CG vectors, the block partial
// sums, the scalars); every value is written before it is read.
int solve_gauss_in(pic_sim *S, double *d, double tol, int max_iter, pic_gauss_out *out, hipStream_t stream)
{
    const pic_config &c = S->cfg;
    const int64_t P = (int64_t)c.nx * c.ny;
    if (!(tol > 0.0)) tol = 1e-12;
    if (max_iter <= 0) max_iter = 20 * (c.nx > c.ny ? c.nx : c.ny) + 100;
    CgScratch w;
    w.x = d;
    w.r = d + P;
    w.p = d + 2 * P;
    w.q = d + 3 * P;
    w.partial = d + 4 * P;
    w.scal = w.partial + kCgPartials;
    int rc = node_density(S, stream);
    if (rc) return rc;
    const CgResult e = cg_project(S->buf.fields, S->rho_now, mean_density(S), 0, c.nx, c.ny, c.dx, c.dy, tol,
                                  max_iter, w, stream);
    if (e.iterations < 0) return PIC_EHIP;
    const CgResult b = cg_project(S->buf.fields, nullptr, 0.0, 1, c.nx, c.ny, c.dx, c.dy, tol, max_iter, w, stream);
    if (b.iterations < 0) return PIC_EHIP;
    rc = hip_ok(hipGetLastError());
    if (rc == PIC_OK) rc = hip_ok(hipStreamSynchronize(stream));
    if (rc) return rc;
    if (out) {
        out->iterations[0] = e.iterations;
        out->iterations[1] = b.iterations;
        out->residual[0] = e.residual;
        out->residual[1] = b.residual;
    }
    S->have_snapshot = false;
    return e.converged && b.converged ? PIC_OK : PIC_ENOCONV;
}


// Kernel arguments of one simulation (identical every step: the sort writes
// the new tile_offset in place).
PushArgs push_args(const pic_sim *S, bool bh)
{
    const pic_config &c = S->cfg;
    PushArgs a;
    memset(&a, 0, sizeof(a));
    a.fld = S->buf.fields;
    a.bh = bh ? S->bh : nullptr;
    a.hdx = (float)(0.5 * c.dt / c.dx);
    a.hdy = (float)(0.5 * c.dt / c.dy);
    a.jtile = S->jtile;
    a.err = S->err;
    a.nx = c.nx;
    a.ny = c.ny;
    a.ntx = S->ntx;
    a.nty = S->nty;
    a.cx = (float)(c.dt / c.dx);
    a.cy = (float)(c.dt / c.dy);
    // accumulator units: the largest particle charge moving one cell (Jx, Jy)
    // or at the speed of light (Jz) is 1 (x 2^30 in fixed point)
    double qmax = 0.0;
    for (int s = 0; s < c.n_species; ++s) qmax = std::max(qmax, fabs(c.species[s].q));
    if (qmax == 0.0) qmax = 1.0;
    const double scale = j_mode(&c) == kJFixed ? (double)kFixedScale : 1.0;
    a.ju[0] = (float)(qmax * c.dx / c.dt / scale);
    a.ju[1] = (float)(qmax * c.dy / c.dt / scale);
    a.ju[2] = (float)(qmax / scale);
    a.n_species = c.n_species;
    a.rebase = S->since_sort == 0 ? 1 : 0;   // batched pushes take theirs from the launch
    a.stg_live = S->stg_live;
    for (int s = 0; s < c.n_species; ++s) {
        const pic_particles &p = S->buf.sp[s];
        SpeciesDev &d = a.sp[s];
        d.cell = S->sp[s].lcell;
        d.x = p.x;
        d.y = p.y;
        d.ux = p.ux;
        d.uy = p.uy;
        d.uz = p.uz;
        d.off = S->sp[s].off;
        d.cnt = S->sp[s].cnt;
        d.leav = S->sp[s].leav;
        d.lrec = S->sp[s].lrec;
        d.fcount = S->sp[s].fcount;
        d.fbase = S->sp[s].fbase;
        d.fhole = S->sp[s].hole;
        d.fsrc = S->sp[s].srec;
        const Parts &g = S->sp[s].stg;
        d.scell = g.cell;
        d.sx = g.x;
        d.sy = g.y;
        d.sux = g.ux;
        d.suy = g.uy;
        d.suz = g.uz;
        d.n = (int32_t)c.species[s].n;
        d.h = (float)(0.5 * c.species[s].qm * c.dt);
        d.fq = (float)(scale * c.species[s].q / qmax);
    }
    return a;
}

float *j_planes(const pic_sim *S) { return S->buf.fields + (int64_t)6 * S->cfg.nx * S->cfg.ny; }

// The filter passes alternate between the J planes and jf; the tile fold
// writes to whichever of the two makes the last pass land in the J planes.
float *j_fold_target(const pic_sim *S) { return (S->cfg.j_filter & 1) ? S->jf : j_planes(S); }

FilterArgs filter_args(const pic_sim *S, int pass)
{
    float *first = j_fold_target(S), *second = first == S->jf ? j_planes(S) : S->jf;
    FilterArgs f;
    f.src = (pass & 1) ? second : first;
    f.dst = (pass & 1) ? first : second;
    f.nx = S->cfg.nx;
    f.ny = S->cfg.ny;
    f.planes = 3;
    return f;
}

JReduceArgs jreduce_args(const pic_sim *S)
{
    JReduceArgs r;
    r.jtile = S->jtile;
    r.J = j_fold_target(S);
    r.nx = S->cfg.nx;
    r.ny = S->cfg.ny;
    r.ntx = S->ntx;
    r.nty = S->nty;
    return r;
}

SortArgs sort_args(const pic_sim *S, bool defer = false)
{
    const pic_config &c = S->cfg;
    SortArgs a;
    memset(&a, 0, sizeof(a));
    a.err = S->err;
    a.stg_live = S->stg_live;
    a.defer = defer ? 1 : 0;
    a.nx = c.nx;
    a.ny = c.ny;
    a.ntx = S->ntx;
    a.nty = S->nty;
    a.tile = S->tile;
    a.n_tiles = S->n_tiles;
    a.n_species = c.n_species;
    for (int s = 0; s < c.n_species; ++s) {
        const pic_particles &p = S->buf.sp[s];
        const auto &P = S->sp[s];
        SortSpecies &d = a.sp[s];
        d.p.cell = P.lcell;
        d.gcell = p.cell;
        d.p.x = p.x;
        d.p.y = p.y;
        d.p.ux = p.ux;
        d.p.uy = p.uy;
        d.p.uz = p.uz;
        d.lrec = P.lrec;
        d.stg = P.stg;
        d.srec = P.srec;
        d.off = P.off;
        d.offp = P.offp;
        d.cnt = P.cnt;
        d.leav = P.leav;
        d.hole = P.hole;
        d.mcount = P.mcount;
        d.fcount = P.fcount;
        d.fbase = P.fbase;
        d.bsum = P.bsum;
        d.n = (int32_t)c.species[s].n;
        d.inj_off = nullptr;
        d.inj_n = 0;
        d.removed = nullptr;
    }
    return a;
}

// fold: J folded from the tile current halos by the E step of the field
// advance (and written to the J planes), else read from the J planes
FieldArgs field_args(const pic_sim *S, bool fold, bool bh)
{
    const pic_config &c = S->cfg;
    FieldArgs f;
    f.fld = S->buf.fields;
    f.jtile = fold ? S->jtile : nullptr;
    f.bh = bh ? S->bh : nullptr;
    f.nx = c.nx;
    f.ny = c.ny;
    f.ntx = S->ntx;
    f.nty = S->nty;
    f.hdx = (float)(0.5 * c.dt / c.dx);
    f.hdy = (float)(0.5 * c.dt / c.dy);
    f.dt = (float)c.dt;
    f.dtdx = (float)(c.dt / c.dx);
    f.dtdy = (float)(c.dt / c.dy);
    return f;
}

}  // namespace

extern "C" {

const char *pic_strerror(int code)
{
    switch (code) {
    case PIC_OK: return "ok";
    case PIC_EINVAL: return "invalid argument";
    case PIC_ECFL: return "time step violates the Courant condition";
    case PIC_ETILE: return "tile size unsupported or does not divide the grid";
    case PIC_EHIP: return "HIP runtime call failed";
    case PIC_EORDER: return "particles not grouped by tile or cell index out of range";
    case PIC_ERANGE: return "a particle moved one cell or more in one step";
    case PIC_ESORT: return "sort consistency check failed";
    case PIC_ECOUNT: return "tile counts do not add up to the particle count";
    case PIC_EOVERFLOW: return "a tile holds 2^31 or more particles (its fixed-point current could overflow)";
    case PIC_ESCRATCH: return "the grid is larger than pic_solve_gauss_noalloc's static scratch holds";
    case PIC_ENOCONV: return "the Poisson iteration did not reach its tolerance";
    default: return "unknown error";
    }
}

int pic_query(const pic_config *cfg, pic_sizes *out)
{
    if (!out) return PIC_EINVAL;
    const int rc = validate(cfg);
    if (rc) return rc;
    const Layout L = make_layout(cfg);
    out->n_tiles = (cfg->nx / cfg->tile) * (cfg->ny / cfg->tile);
    out->field_bytes = (size_t)9 * cfg->nx * cfg->ny * sizeof(float);
    out->work_bytes = L.total;
    return PIC_OK;
}

namespace {

// tile_offset of every species from its particle cells (which must be grouped
// by tile); synchronises and reports PIC_EORDER / PIC_ECOUNT.
// The stable radix regrouping of species s, on the per-particle scratch of
// the in-place sort and the leaver copies (free at initialisation, and after a
// push when the full re-sort replaces the in-place one) and, for the
// histogram, the leaver copies' cell array (n >= its size) or the tile
// current halos (consumed by then: pic_step folds them before a full
// re-sort, on the same stream).
TileSortArgs tile_sort_args(pic_sim *S, int s)
{
    auto &P = S->sp[s];
    const pic_particles &b = S->buf.sp[s];
    const int n = (int)S->cfg.species[s].n;
    TileSortArgs t;
    t.p = GParts{b.cell, b.x, b.y, b.ux, b.uy, b.uz};
    t.tmp = P.lp;
    t.key[0] = (uint32_t *)P.hole;
    t.key[1] = P.leav;
    // scratch: the in-place sort's staging records (8 n words)
    t.val[0] = (uint32_t *)P.srec;
    t.val[1] = (uint32_t *)P.srec + n;
    t.hist = tile_sort_hist_entries(n) <= n ? P.lp.cell : (int32_t *)S->jtile;
    t.n = n;
    t.tile = S->cfg.tile;
    t.ntx = S->ntx;
    t.n_tiles = S->n_tiles;
    return t;
}

// tile_offset of every species from its particles, grouping them by tile
// first (stable radix sort on the device) if they arrive in another order.
// PIC_EORDER if a cell is outside the grid.  The sort's scratch is the
// per-particle workspace of the sort and the leaver copies, free before the
// first push.
int build_tiles(pic_sim *S, hipStream_t stream)
{
    const pic_config &c = S->cfg;
    int rc = PIC_OK;
    for (int s = 0; s < c.n_species && rc == PIC_OK; ++s) {
        auto &P = S->sp[s];
        const int n = (int)c.species[s].n;
        for (int attempt = 0; attempt < 2 && rc == PIC_OK; ++attempt) {
            launch_init_tiles(S->buf.sp[s].cell, n, c.nx, c.ny, c.tile, S->ntx, S->n_tiles, P.off, S->err, stream);
            rc = hip_ok(hipGetLastError());
            int h = 0;
            if (rc == PIC_OK) rc = read_flags(S, stream, &h);
            if (rc) break;
            if (h & kErrOrder) return PIC_EORDER;
            if (!(h & kErrGroup)) break;
            if (attempt == 1) return PIC_ESORT;   // still not grouped after the sort
            launch_tile_sort(tile_sort_args(S, s), stream);
            rc = hip_ok(hipGetLastError());
        }
        if (rc == PIC_OK) launch_localize(S->buf.sp[s].cell, P.lcell, n, c.tile, stream);
        if (rc == PIC_OK) rc = hip_ok(hipMemsetAsync(P.mcount, 0, (size_t)S->n_tiles * sizeof(int32_t), stream));
        if (rc == PIC_OK) rc = hip_ok(hipMemsetAsync(P.fcount, 0, (size_t)S->n_tiles * sizeof(int32_t), stream));
    }
    if (rc == PIC_OK) rc = read_errors(S, stream);
    return rc;
}

}  // namespace

namespace {
// with_side: create pic_step's second stream (the members of a batch have
// none: the batch forks its own step)
int init_sim(const pic_config *cfg, const pic_buffers *bufs, hipStream_t stream, pic_sim **out, bool with_side);
}  // namespace

int pic_init(const pic_config *cfg, const pic_buffers *bufs, hipStream_t stream, pic_sim **out)
{
    return init_sim(cfg, bufs, stream, out, true);
}

}  // extern "C"

namespace {

int init_sim(const pic_config *cfg, const pic_buffers *bufs, hipStream_t stream, pic_sim **out, bool with_side)
{
    if (!out || !bufs) return PIC_EINVAL;
    *out = nullptr;
    int rc = validate(cfg);
    if (rc) return rc;
    const Layout L = make_layout(cfg);
    if (!bufs->fields || !bufs->work || bufs->work_bytes < L.total) return PIC_EINVAL;
    if (((uintptr_t)bufs->work) % kAlign) return PIC_EINVAL;
    for (int s = 0; s < cfg->n_species; ++s) {
        const pic_particles &p = bufs->sp[s];
        if (cfg->species[s].n > 0 && (!p.cell || !p.x || !p.y || !p.ux || !p.uy || !p.uz)) return PIC_EINVAL;
    }

    pic_sim *S = new (std::nothrow) pic_sim();
    if (!S) return PIC_EINVAL;
    S->cfg = *cfg;
    S->buf = *bufs;
    S->tile = cfg->tile;
    S->ntx = cfg->nx / cfg->tile;
    S->nty = cfg->ny / cfg->tile;
    S->n_tiles = S->ntx * S->nty;
    S->replicas = cfg->j_replicas ? cfg->j_replicas : default_replicas(cfg);
    char *w = (char *)bufs->work;
    S->work = w;
    S->err = (int *)(w + L.err);
    S->stg_live = (int *)(w + L.stg_live);
    S->dacc = (double *)(w + L.dacc);
    S->cacc = (unsigned long long *)(w + L.cacc);
    S->jtile = (float *)(w + L.jtile);
    S->bh = (float *)(w + L.bh);
    S->rho_prev = (double *)(w + L.rho_prev);
    S->rho_now = (double *)(w + L.rho_now);
    S->jf = cfg->j_filter > 0 ? (float *)(w + L.jf) : nullptr;
    S->rho_tmp = cfg->j_filter > 0 ? (double *)(w + L.rho_tmp) : nullptr;
    const bool window = (cfg->flags & PIC_FLAG_MOVING_WINDOW) != 0;
    S->wrem = window ? (int32_t *)(w + L.wrem) : nullptr;
    S->origin = 0;
    S->cadence = cadence_of(cfg);
    S->halo = halo_of(cfg);
    S->since_sort = 0;
    for (int s = 0; s < cfg->n_species; ++s) {
        auto &P = S->sp[s];
        P.off = (int32_t *)(w + L.off[s][0]);
        P.offp = (int32_t *)(w + L.off[s][1]);
        P.cnt = (int32_t *)(w + L.cnt[s]);
        P.leav = (uint32_t *)(w + L.leav[s]);
        P.hole = (int32_t *)(w + L.hole[s]);
        P.lcell = (int16_t *)(w + L.lcell[s]);
        auto parts_at = [&](const size_t *o) {
            Parts q;
            q.cell = (int16_t *)(w + o[0]);
            q.x = (float *)(w + o[1]);
            q.y = (float *)(w + o[2]);
            q.ux = (float *)(w + o[3]);
            q.uy = (float *)(w + o[4]);
            q.uz = (float *)(w + o[5]);
            return q;
        };
        const bool motion = (cfg->flags & PIC_FLAG_MOTION_SORT) != 0;
        P.stg = motion ? parts_at(L.stg[s]) : Parts{};
        P.srec = (LeaverRec *)(w + L.srec[s]);
        P.lrec = (LeaverRec *)(w + L.lrec[s]);
        {
            size_t o[6];
            const size_t n = (size_t)(cfg->species[s].cap ? cfg->species[s].cap : cfg->species[s].n);
            for (int k = 0; k < 6; ++k) o[k] = L.lrec[s] + align_up((size_t)k * n * 4);
            P.lp = GParts{(int32_t *)(w + o[0]), (float *)(w + o[1]), (float *)(w + o[2]), (float *)(w + o[3]),
                          (float *)(w + o[4]), (float *)(w + o[5])};
        }
        P.mcount = (int32_t *)(w + L.mcount[s]);
        P.fcount = (int32_t *)(w + L.fcount[s]);
        P.fbase = (int32_t *)(w + L.fbase[s]);
        P.bsum = (int32_t *)(w + L.bsum[s]);
        P.inj_off = window ? (int32_t *)(w + L.inj_off[s]) : nullptr;
        S->cap[s] = cfg->species[s].cap ? cfg->species[s].cap : cfg->species[s].n;
    }

    rc = hip_ok(hipGetDevice(&S->device));
    if (rc == PIC_OK) {
        // set-up of pic_solve_gauss_noalloc on this device (a failure here is
        // reported by that call, which looks the address up again)
        void *unused = nullptr;
        (void)scratch_address(S->device, &unused);
    }
    if (rc == PIC_OK) rc = hip_ok(hipMemsetAsync(S->err, 0, 64, stream));
    if (rc == PIC_OK) rc = hip_ok(hipMemsetAsync(S->stg_live, 0, sizeof(int), stream));
    if (rc == PIC_OK) rc = build_tiles(S, stream);
    if (with_side) {
        // default priority, like every stream of the library's callers
        if (rc == PIC_OK) rc = hip_ok(hipStreamCreateWithFlags(&S->side, hipStreamNonBlocking));
        if (rc == PIC_OK) rc = hip_ok(hipEventCreateWithFlags(&S->ev_fork, hipEventDisableTiming));
        if (rc == PIC_OK) rc = hip_ok(hipEventCreateWithFlags(&S->ev_join, hipEventDisableTiming));
    }
    if (rc != PIC_OK) {
        release_side(S);
        delete S;
        return rc;
    }
    *out = S;
    return PIC_OK;
}

}  // namespace

extern "C" {


namespace {

// Whether pic_step's motion-class sort leaves its copy back to the next push
// (which then reads the staging arrays): the push is built for that with
// the default current and deposit.
bool motion_deferrable(const pic_sim *S)
{
    return (S->cfg.flags & PIC_FLAG_MOTION_SORT) && j_mode(&S->cfg) == kJFixed && S->replicas == 1 &&
           d_mode(&S->cfg) == kDepVB;
}

// The push kernel alone (steps a1-a7 up to the per-tile current halos); with
// bh, it also forms the field advance's first half step (pic_step).
int push_only(pic_sim *S, hipStream_t stream, bool bh)
{
    // a particle may stray at most sort_every - 1 cells from its tile before a push
    if (S->since_sort >= S->cadence) return PIC_EORDER;
    const PushArgs a = push_args(S, bh);
    const bool ms = motion_deferrable(S);
    {
        Timed t(S, PIC_KERNEL_PUSH, stream);
        launch_push_deposit(S->tile, S->replicas, j_mode(&S->cfg), d_mode(&S->cfg), S->halo, ppl_of(&S->cfg), a,
                            S->n_tiles, ms, stream);
    }
    // the push has taken the particles from wherever they were: from now on
    // the particle arrays hold them
    if (ms) launch_set_int(S->stg_live, 0, stream);
    S->since_sort += 1;
    return hip_ok(hipGetLastError());
}

// The fold of the tile current halos into J, then the optional filter passes.
int fold_current(pic_sim *S, hipStream_t stream);

// The field half of a step after a push that formed the first B half step:
// the J fold (and the filter), then the E step and the second B half step --
// the fold done by the E step when there is no filter (the same J, bit for
// bit: both use fold_node).  The same fields as pic_field_advance, bit for
// bit: the push's half step uses the same per-cell function.
int field_half(pic_sim *S, hipStream_t stream)
{
    const bool fold = S->cfg.j_filter == 0;
    if (!fold) {
        const int rc = fold_current(S, stream);
        if (rc) return rc;
    }
    Timed t(S, PIC_KERNEL_FIELD, stream);
    launch_field_advance(field_args(S, fold, true), S->tile, S->halo, stream);
    return hip_ok(hipGetLastError());
}

int fold_current(pic_sim *S, hipStream_t stream)
{
    {
        Timed t(S, PIC_KERNEL_JREDUCE, stream);
        launch_j_reduce(S->tile, S->halo, jreduce_args(S), stream);
    }
    for (int p = 0; p < S->cfg.j_filter; ++p) {
        Timed t(S, PIC_KERNEL_FILTER, stream);
        launch_filter(filter_args(S, p), false, stream);
    }
    return hip_ok(hipGetLastError());
}

}  // namespace

int pic_push_deposit(pic_sim *S, hipStream_t stream)
{
    if (!S) return PIC_EINVAL;
    int rc = push_only(S, stream, false);
    if (rc == PIC_OK) rc = fold_current(S, stream);
    return rc;
}

// The alternative sort (PIC_FLAG_MOTION_SORT): the motion-class sort --
// recount and scan as for the in-place sort, then every particle into the
// staging arrays at its slot in the (new tile, motion class, old slot) order
// (timed as plan), and the staging arrays copied back (timed as scatter) --
// or, deferred (pic_step), read from there by the next push.
static int motion_sort(pic_sim *S, hipStream_t stream, bool defer)
{
    const SortArgs a = sort_args(S, defer);
    {
        Timed t(S, PIC_KERNEL_SORT_SCAN, stream);
        launch_sort_scan(a, S->n_tiles, stream);
    }
    {
        Timed t(S, PIC_KERNEL_SORT_PLAN, stream);
        launch_motion_scatter(a, S->n_tiles, stream);
    }
    if (!defer) {
        Timed t(S, PIC_KERNEL_SORT_SCATTER, stream);
        launch_motion_copy(a, S->n_tiles, stream);
    }
    return hip_ok(hipGetLastError());
}

// The sort after a push; defer: the in-place sort leaves its hole fill to
// the next push (pic_step), which streams those slots anyway.
static int sort_after_push(pic_sim *S, hipStream_t stream, bool defer)
{
    if (S->since_sort == 0) return PIC_OK;   // already sorted: the count records are spent
    S->since_sort = 0;
    if (S->cfg.flags & PIC_FLAG_MOTION_SORT) return motion_sort(S, stream, defer && motion_deferrable(S));
    const SortArgs a = sort_args(S, defer);
    {
        Timed t(S, PIC_KERNEL_SORT_SCAN, stream);
        launch_sort_scan(a, S->n_tiles, stream);
    }
    {
        Timed t(S, PIC_KERNEL_SORT_PLAN, stream);
        launch_sort_plan(a, S->n_tiles, stream);
    }
    if (!defer) {   // deferred: the next push places the movers
        Timed t(S, PIC_KERNEL_SORT_SCATTER, stream);
        launch_sort_scatter(a, S->n_tiles, stream);
    }
    return hip_ok(hipGetLastError());
}

// A fill (or the motion-class sort's copy back) left pending by pic_step's
// sort, done before anything but a push reads the particle arrays, and
// (publish) the whole-grid cells written into the caller's cell arrays from
// the tile-relative ones the kernels keep.  Always launched: the device fill
// counts and flag, not the host, know whether anything is pending (replays
// of a captured step run no host code); a tile with no fill costs one read.
static int settle(pic_sim *S, hipStream_t stream, bool publish = true)
{
    const SortArgs a = sort_args(S);
    if (motion_deferrable(S)) launch_motion_copy_live(a, S->n_tiles, stream);   // a copy back left pending
    launch_fill(a, S->n_tiles, stream);
    if (publish) launch_publish(a, S->n_tiles, S->since_sort == 0, stream);
    return hip_ok(hipGetLastError());
}

int pic_sort(pic_sim *S, hipStream_t stream)
{
    if (!S) return PIC_EINVAL;
    return sort_after_push(S, stream, false);
}

int pic_sync(pic_sim *S, hipStream_t stream)
{
    if (!S) return PIC_EINVAL;
    return settle(S, stream);
}

int pic_field_advance(pic_sim *S, hipStream_t stream)
{
    if (!S) return PIC_EINVAL;
    Timed t(S, PIC_KERNEL_FIELD, stream);
    launch_field_advance(field_args(S, false, false), S->tile, S->halo, stream);
    return hip_ok(hipGetLastError());
}

int pic_move_window(pic_sim *S, const pic_particles *inject, const int64_t *n_inject, hipStream_t stream)
{
    if (!S || !(S->cfg.flags & PIC_FLAG_MOVING_WINDOW)) return PIC_EINVAL;
    if (S->since_sort != 0) return PIC_EORDER;   // the last push is not sorted yet
    if (const int rs = settle(S, stream, false)) return rs;   // the window reads the tile-relative cells
    pic_config &c = S->cfg;
    int64_t k[kMaxSpecies] = {};
    for (int s = 0; s < c.n_species; ++s) {
        k[s] = n_inject ? n_inject[s] : 0;
        if (k[s] < 0 || c.species[s].n + k[s] > S->cap[s]) return PIC_EINVAL;
        if (k[s] > 0) {
            if (!inject) return PIC_EINVAL;
            const pic_particles &q = inject[s];
            if (!q.cell || !q.x || !q.y || !q.ux || !q.uy || !q.uz) return PIC_EINVAL;
        }
    }
    // array column of window column 0 now, and of window column nx - 1 after the move
    const int col = S->origin;
    SortArgs a = sort_args(S);
    a.rebase = 1;   // sorted: no push since the last sort
    int rc = PIC_OK;
    // 1. the new particles into the unused slots after the existing ones, their
    //    cells moved to array column col, and checked (window column nx - 1,
    //    grouped by tile) before anything changes
    for (int s = 0; s < c.n_species && rc == PIC_OK; ++s) {
        if (k[s] == 0) continue;
        const pic_particles &p = S->buf.sp[s];
        auto &P = S->sp[s];
        const size_t n0 = (size_t)c.species[s].n, bytes = (size_t)k[s] * 4;
        const pic_particles &q = inject[s];
        void *const dst[5] = {p.x + n0, p.y + n0, p.ux + n0, p.uy + n0, p.uz + n0};
        const void *const src[5] = {q.x, q.y, q.ux, q.uy, q.uz};
        for (int f = 0; f < 5 && rc == PIC_OK; ++f)
            rc = hip_ok(hipMemcpyAsync(dst[f], src[f], bytes, hipMemcpyDeviceToDevice, stream));
        if (rc) break;
        launch_place_new(q.cell, p.cell + n0, P.lcell + n0, (int)k[s], c.nx, c.ny, col, c.tile, S->err, stream);
        launch_init_tiles(p.cell + n0, (int32_t)k[s], c.nx, c.ny, c.tile, S->ntx, S->n_tiles, P.inj_off, S->err,
                          stream);
        a.sp[s].inj_off = P.inj_off;
        a.sp[s].inj_n = (int32_t)k[s];
    }
    if (rc == PIC_OK) rc = hip_ok(hipGetLastError());
    if (rc == PIC_OK) rc = read_errors(S, stream);
    if (rc) return rc;
    // 2. E and B of the column that becomes window column nx - 1
    launch_zero_column(S->buf.fields, c.nx, c.ny, col, stream);
    launch_zero_i32(S->wrem, kMaxSpecies, stream);
    // 3. its particles leave: leaver lists and count records for the sort
    for (int s = 0; s < c.n_species && rc == PIC_OK; ++s) {
        auto &P = S->sp[s];
        WindowSpecies ws;
        ws.p = a.sp[s].p;
        ws.off = P.off;
        ws.cnt = P.cnt;
        ws.leav = P.leav;
        ws.removed = S->wrem + s;
        launch_window_remove(S->tile, ws, S->ntx, S->nty, S->n_tiles, col, stream);
        a.sp[s].removed = S->wrem + s;
    }
    if (rc == PIC_OK) rc = hip_ok(hipGetLastError());
    if (rc) return rc;
    // 4. the canonical re-sort, the new particles taken as appended
    launch_sort_scan(a, S->n_tiles, stream);
    launch_sort_plan(a, S->n_tiles, stream);
    launch_sort_scatter(a, S->n_tiles, stream);
    rc = hip_ok(hipGetLastError());
    // the new counts
    int32_t nn[kMaxSpecies] = {};
    for (int s = 0; s < c.n_species && rc == PIC_OK; ++s)
        rc = hip_ok(hipMemcpyAsync(&nn[s], S->sp[s].off + S->n_tiles, sizeof(int32_t), hipMemcpyDeviceToHost,
                                   stream));
    if (rc == PIC_OK) rc = hip_ok(hipStreamSynchronize(stream));
    if (rc) return rc;
    rc = read_errors(S, stream);
    if (rc) return rc;
    for (int s = 0; s < c.n_species; ++s) c.species[s].n = nn[s];
    S->origin = col + 1 == c.nx ? 0 : col + 1;
    S->have_snapshot = false;
    return PIC_OK;
}

int pic_get_window_origin(pic_sim *S, int32_t *origin)
{
    if (!S || !origin) return PIC_EINVAL;
    *origin = S->origin;
    return PIC_OK;
}

int pic_solve_gauss(pic_sim *S, void *work, size_t work_bytes, double tol, int max_iter, pic_gauss_out *out,
                    hipStream_t stream)
{
    if (!S || !work || ((uintptr_t)work) % kAlign) return PIC_EINVAL;
    if (work_bytes < PIC_GAUSS_SCRATCH_BYTES(S->cfg.nx, S->cfg.ny)) return PIC_EINVAL;
    if (const int rs = settle(S, stream)) return rs;   // the density reads the particles
    return solve_gauss_in(S, (double *)work, tol, max_iter, out, stream);
}

int pic_solve_gauss_noalloc(pic_sim *S, double tol, int max_iter, pic_gauss_out *out, hipStream_t stream)
{
    if (!S) return PIC_EINVAL;
    if ((int64_t)S->cfg.nx * S->cfg.ny > PIC_GAUSS_NOALLOC_MAX_CELLS) return PIC_ESCRATCH;
    int dev = -1;
    int rc = hip_ok(hipGetDevice(&dev));
    if (rc) return rc;
    if (dev != S->device) return PIC_EINVAL;
    void *p = nullptr;
    rc = scratch_address(dev, &p);
    if (rc == PIC_OK) rc = settle(S, stream);   // the density reads the particles
    if (rc) return rc;
    return solve_gauss_in(S, (double *)p, tol, max_iter, out, stream);
}

int pic_get_counts(pic_sim *S, int64_t *counts)
{
    if (!S || !counts) return PIC_EINVAL;
    for (int s = 0; s < S->cfg.n_species; ++s) counts[s] = S->cfg.species[s].n;
    return PIC_OK;
}

int pic_step(pic_sim *S, hipStream_t stream)
{
    if (!S) return PIC_EINVAL;
    int rc = push_only(S, stream, true);
    if (rc) return rc;
    // Unforked: no sort this step, or no second stream
    if (S->since_sort < S->cadence || !S->side) {
        if (S->since_sort >= S->cadence) rc = sort_after_push(S, stream, true);
        if (rc == PIC_OK) rc = field_half(S, stream);
        return rc;
    }
    // Once the push is done, the sort (particles, count records, leaver
    // lists) and the field half (tile current halos, J, E, B) touch disjoint
    // data: the field half runs on the second stream, beside the sort, and
    // the caller's stream waits for it before anything later.  Both halves
    // are small, latency-bound kernels, so they overlap well.
    rc = hip_ok(hipEventRecord(S->ev_fork, stream));
    if (rc) return rc;
    rc = hip_ok(hipStreamWaitEvent(S->side, S->ev_fork, 0));
    if (rc) return rc;
    int rf = field_half(S, S->side);
    const int rj = hip_ok(hipEventRecord(S->ev_join, S->side));
    rc = sort_after_push(S, stream, true);
    // the join is enqueued whatever happened above, so the caller's stream
    // never runs ahead of work already on the second stream
    const int rw = rj == PIC_OK ? hip_ok(hipStreamWaitEvent(stream, S->ev_join, 0)) : rj;
    return rc ? rc : (rf ? rf : rw);
}

int pic_check(pic_sim *S, hipStream_t stream)
{
    if (!S) return PIC_EINVAL;
    return read_errors(S, stream);
}

int pic_diag(pic_sim *S, unsigned what, pic_diag_out *out, hipStream_t stream)
{
    if (!S || !out) return PIC_EINVAL;
    memset(out, 0, sizeof(*out));
    const pic_config &c = S->cfg;
    const int64_t plane = (int64_t)c.nx * c.ny;
    if ((what & PIC_DIAG_CONTINUITY) && !S->have_snapshot) return PIC_EINVAL;
    int rc = settle(S, stream);
    if (rc == PIC_OK) rc = hip_ok(hipMemsetAsync(S->dacc, 0, 32 * sizeof(double), stream));
    if (rc == PIC_OK) rc = hip_ok(hipMemsetAsync(S->cacc, 0, 8 * sizeof(unsigned long long), stream));
    if (rc) return rc;
    if (what & PIC_DIAG_ENERGY) {
        launch_diag_field_energy(S->buf.fields, plane, S->dacc, stream);
        for (int s = 0; s < c.n_species; ++s) launch_diag_kinetic(diag_species(S, s), S->dacc + 2 + s, stream);
    }
    if (what & (PIC_DIAG_RHO_SNAPSHOT | PIC_DIAG_CONTINUITY | PIC_DIAG_GAUSS)) {
        rc = node_density(S, stream);
        if (rc) return rc;
    }
    if (what & PIC_DIAG_CONTINUITY)
        launch_diag_continuity(S->rho_prev, S->rho_now, S->buf.fields + 6 * plane, c.nx, c.ny, c.dt, c.dx, c.dy,
                               S->dacc + 8, stream);
    if (what & PIC_DIAG_GAUSS)
        launch_diag_gauss(S->buf.fields, S->rho_now, mean_density(S), c.nx, c.ny, c.dx, c.dy, S->dacc + 10, stream);
    double dh[32];
    unsigned long long ch[8 * kMaxSpecies];
    rc = hip_ok(hipMemcpyAsync(dh, S->dacc, sizeof(dh), hipMemcpyDeviceToHost, stream));
    if (rc == PIC_OK && (what & PIC_DIAG_COUNTS)) {
        for (int s = 0; s < c.n_species && rc == PIC_OK; ++s) {
            rc = hip_ok(hipMemsetAsync(S->cacc, 0, 2 * sizeof(unsigned long long), stream));
            if (rc) break;
            launch_diag_counts(S->sp[s].cnt, S->sp[s].mcount, S->n_tiles, S->cacc, stream);
            rc = hip_ok(hipMemcpyAsync(ch + 2 * s, S->cacc, 2 * sizeof(unsigned long long),
                                       hipMemcpyDeviceToHost, stream));
            if (rc == PIC_OK) rc = hip_ok(hipStreamSynchronize(stream));
        }
    }
    if (rc == PIC_OK) rc = hip_ok(hipStreamSynchronize(stream));
    if (rc) return rc;
    if (what & PIC_DIAG_ENERGY) {
        const double dA = c.dx * c.dy;
        out->u_e = 0.5 * dA * dh[0];
        out->u_b = 0.5 * dA * dh[1];
        for (int s = 0; s < c.n_species; ++s)
            out->u_k[s] = dA * (c.species[s].q / c.species[s].qm) * dh[2 + s];
    }
    if (what & PIC_DIAG_CONTINUITY) {
        out->continuity_max = dh[8];
        out->rho_max = dh[9];
    }
    if (what & PIC_DIAG_GAUSS) {
        out->gauss_max = dh[10];
        out->divb_max = dh[11];
    }
    if (what & PIC_DIAG_COUNTS)
        for (int s = 0; s < c.n_species; ++s) {
            out->leavers[s] = (int64_t)ch[2 * s];
            out->movers[s] = (int64_t)ch[2 * s + 1];
        }
    if (what & (PIC_DIAG_RHO_SNAPSHOT | PIC_DIAG_CONTINUITY)) {
        std::swap(S->rho_prev, S->rho_now);
        S->have_snapshot = true;
    }
    return read_errors(S, stream);
}

namespace {

// one host <-> device copy of each particle array of species s
int copy_particles(pic_sim *S, int s, const pic_particles &host, bool to_host, hipStream_t stream)
{
    const pic_particles &dev = S->buf.sp[s];
    const size_t n = (size_t)S->cfg.species[s].n;
    void *const hp[6] = {host.cell, host.x, host.y, host.ux, host.uy, host.uz};
    void *const dp[6] = {dev.cell, dev.x, dev.y, dev.ux, dev.uy, dev.uz};
    int rc = PIC_OK;
    for (int k = 0; k < 6 && rc == PIC_OK && n > 0; ++k) {
        if (!hp[k]) {
            if (to_host) continue;
            return PIC_EINVAL;
        }
        rc = to_host ? hip_ok(hipMemcpyAsync(hp[k], dp[k], 4 * n, hipMemcpyDeviceToHost, stream))
                     : hip_ok(hipMemcpyAsync(dp[k], hp[k], 4 * n, hipMemcpyHostToDevice, stream));
    }
    return rc;
}

}  // namespace

int pic_get_state(pic_sim *S, pic_host_state *out, hipStream_t stream)
{
    if (!S || !out) return PIC_EINVAL;
    const size_t fbytes = 9 * sizeof(float) * (size_t)S->cfg.nx * S->cfg.ny;
    int rc = settle(S, stream);
    if (out->fields) rc = hip_ok(hipMemcpyAsync(out->fields, S->buf.fields, fbytes, hipMemcpyDeviceToHost, stream));
    for (int s = 0; s < S->cfg.n_species && rc == PIC_OK; ++s) rc = copy_particles(S, s, out->sp[s], true, stream);
    if (rc == PIC_OK) rc = hip_ok(hipStreamSynchronize(stream));
    if (rc == PIC_OK) {
        out->window_origin = S->origin;
        for (int s = 0; s < PIC_MAX_SPECIES; ++s) out->n[s] = s < S->cfg.n_species ? S->cfg.species[s].n : 0;
    }
    return rc;
}

int pic_set_state(pic_sim *S, const pic_host_state *in, hipStream_t stream)
{
    if (!S || !in || !in->fields) return PIC_EINVAL;
    const bool window = (S->cfg.flags & PIC_FLAG_MOVING_WINDOW) != 0;
    if (in->window_origin < 0 || in->window_origin >= S->cfg.nx || (!window && in->window_origin != 0))
        return PIC_EINVAL;
    for (int s = 0; s < S->cfg.n_species; ++s) {
        const pic_particles &p = in->sp[s];
        const int64_t n = in->n[s];
        if (n < 0 || n > S->cap[s] || (!window && n != S->cfg.species[s].n)) return PIC_EINVAL;
        if (n > 0 && (!p.cell || !p.x || !p.y || !p.ux || !p.uy || !p.uz)) return PIC_EINVAL;
    }
    for (int s = 0; s < S->cfg.n_species; ++s) S->cfg.species[s].n = in->n[s];
    const size_t fbytes = 9 * sizeof(float) * (size_t)S->cfg.nx * S->cfg.ny;
    int rc = hip_ok(hipMemcpyAsync(S->buf.fields, in->fields, fbytes, hipMemcpyHostToDevice, stream));
    for (int s = 0; s < S->cfg.n_species && rc == PIC_OK; ++s) rc = copy_particles(S, s, in->sp[s], false, stream);
    S->have_snapshot = false;
    S->since_sort = 0;
    if (rc == PIC_OK) launch_set_int(S->stg_live, 0, stream);   // the new particles are in the arrays
    if (rc == PIC_OK) rc = build_tiles(S, stream);
    if (rc == PIC_OK) S->origin = in->window_origin;
    return rc;
}

int pic_get_tile_offsets(pic_sim *S, int species, int32_t *host_out, hipStream_t stream)
{
    if (!S || !host_out || species < 0 || species >= S->cfg.n_species) return PIC_EINVAL;
    const auto &P = S->sp[species];
    int rc = hip_ok(hipMemcpyAsync(host_out, P.off, (size_t)(S->n_tiles + 1) * sizeof(int32_t),
                                   hipMemcpyDeviceToHost, stream));
    if (rc == PIC_OK) rc = hip_ok(hipStreamSynchronize(stream));
    return rc;
}

int pic_set_timing_mask(pic_sim *S, unsigned mask)
{
    if (!S) return PIC_EINVAL;
    for (int k = 0; k < PIC_N_KERNELS; ++k) {
        for (auto &pr : S->pending[k]) {
            (void)hipEventSynchronize(pr.second);
            S->pool.push_back(pr.first);
            S->pool.push_back(pr.second);
        }
        S->pending[k].clear();
        S->ms[k] = 0.0;
        S->launches[k] = 0;
    }
    S->timing_mask = mask & ((1u << PIC_N_KERNELS) - 1u);
    S->timing = S->timing_mask != 0;
    return PIC_OK;
}

int pic_set_timing(pic_sim *S, int enable)
{
    return pic_set_timing_mask(S, enable ? (1u << PIC_N_KERNELS) - 1u : 0u);
}

int pic_get_timing(pic_sim *S, pic_timing_out *out)
{
    if (!S || !out) return PIC_EINVAL;
    int rc = PIC_OK;
    for (int k = 0; k < PIC_N_KERNELS; ++k) {
        for (auto &pr : S->pending[k]) {
            if (hipEventSynchronize(pr.second) != hipSuccess) rc = PIC_EHIP;
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, pr.first, pr.second) != hipSuccess) rc = PIC_EHIP;
            S->ms[k] += ms;
            S->launches[k] += 1;
            S->pool.push_back(pr.first);
            S->pool.push_back(pr.second);
        }
        S->pending[k].clear();
        out->ms_total[k] = S->ms[k];
        out->launches[k] = S->launches[k];
    }
    return rc;
}

void pic_destroy(pic_sim *S)
{
    if (!S) return;
    for (int k = 0; k < PIC_N_KERNELS; ++k)
        for (auto &pr : S->pending[k]) {
            (void)hipEventSynchronize(pr.second);
            S->pool.push_back(pr.first);
            S->pool.push_back(pr.second);
        }
    for (hipEvent_t e : S->pool) (void)hipEventDestroy(e);
    release_side(S);
    delete S;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched mode
// ---------------------------------------------------------------------------

struct pic_batch {
    std::vector<pic_sim *> sims;
    int tile, replicas, jm, dm;
    int cadence; // sort cadence shared by the members
    int halo;    // the push kernel's halo pad
    int ppl;     // particles per lane of the push loop, shared by the members
    int phase;   // steps since the members were last sorted
    char *dev;
    // device tables
    PushArgs *d_push;
    JReduceArgs *d_jr;
    SortArgs *d_sort;
    FieldArgs *d_field;
    FilterArgs *d_filter;   // 2 n: the even passes, then the odd passes
    int j_filter;
    int4 *push_items, *node_items, *count_items, *scan_items, *plan_items;
    int n_push, n_node, n_count, n_scan, n_plan;
    int max_blocks;   // the most scan blocks of one member
    hipGraph_t graph;
    hipGraphExec_t exec;
    // the field half of a sorting step runs here beside the sort (as in pic_step)
    hipStream_t side;
    hipEvent_t ev_fork, ev_join;
};

namespace {

struct BatchLayout {
    size_t d_push, d_jr, d_sort, d_field, d_filter, push_items, node_items, count_items, scan_items, plan_items,
        total;
    int n_push, n_node, n_count, n_scan, n_plan;
};

int batch_validate(int n, const pic_config *cfgs)
{
    if (n < 1 || !cfgs) return PIC_EINVAL;
    for (int i = 0; i < n; ++i) {
        const int rc = validate(&cfgs[i]);
        if (rc) return rc;
        if (cfgs[i].tile != cfgs[0].tile || cfgs[i].flags != cfgs[0].flags ||
            cfgs[i].j_replicas != cfgs[0].j_replicas || cfgs[i].j_filter != cfgs[0].j_filter ||
            halo_of(&cfgs[i]) != halo_of(&cfgs[0]) || ppl_of(&cfgs[i]) != ppl_of(&cfgs[0]))
            return PIC_EINVAL;
        if (cfgs[i].flags & PIC_FLAG_MOVING_WINDOW) return PIC_EINVAL;   // member counts are fixed
    }
    return PIC_OK;
}

BatchLayout batch_layout(int n, const pic_config *cfgs)
{
    BatchLayout L;
    L.n_push = L.n_node = L.n_count = L.n_scan = L.n_plan = 0;
    for (int i = 0; i < n; ++i) {
        const pic_config &c = cfgs[i];
        const int nt = (c.nx / c.tile) * (c.ny / c.tile);
        L.n_push += nt;
        L.n_node += ((c.nx + 63) / 64) * ((c.ny + 3) / 4);
        L.n_count += c.n_species * ((nt + kScanBlock - 1) / kScanBlock);
        L.n_scan += c.n_species;
        L.n_plan += c.n_species * ((nt + kSortWaves - 1) / kSortWaves);
    }
    size_t p = 0;
    auto take = [&](size_t bytes) {
        const size_t at = p;
        p = align_up(p + std::max<size_t>(bytes, 1));
        return at;
    };
    L.d_push = take(n * sizeof(PushArgs));
    L.d_jr = take(n * sizeof(JReduceArgs));
    L.d_sort = take(n * sizeof(SortArgs));
    L.d_field = take(n * sizeof(FieldArgs));
    L.d_filter = take(2 * n * sizeof(FilterArgs));
    L.push_items = take(L.n_push * sizeof(int4));
    L.node_items = take(L.n_node * sizeof(int4));
    L.count_items = take(L.n_count * sizeof(int4));
    L.scan_items = take(L.n_scan * sizeof(int4));
    L.plan_items = take(L.n_plan * sizeof(int4));
    L.total = p;
    return L;
}

// One step of every member; the sort only when `sort` is set (the last step
// of a cadence cycle); rebase: the first step after a sort.
void batch_enqueue_step(pic_batch *b, bool sort, bool rebase, hipStream_t stream)
{
    {
        // member 0's event timing, if on, times the batch's push launch
        Timed t(b->sims[0], PIC_KERNEL_PUSH, stream);
        launch_push_batch(b->tile, b->replicas, b->jm, b->dm, b->halo, b->ppl, b->d_push, b->push_items,
                          b->n_push, rebase, stream);
    }
    // with a sort, the field half goes to the second stream (disjoint data)
    const bool fork = sort && b->side;
    hipStream_t fs = stream;
    if (fork) {
        (void)hipEventRecord(b->ev_fork, stream);
        (void)hipStreamWaitEvent(b->side, b->ev_fork, 0);
        fs = b->side;
    }
    // the J fold, fused into the field advance when there is no filter
    if (b->j_filter > 0) {
        launch_j_reduce_batch(b->tile, b->halo, b->d_jr, b->node_items, b->n_node, fs);
        for (int p = 0; p < b->j_filter; ++p)
            launch_filter_batch(b->d_filter + (p & 1) * b->sims.size(), b->node_items, b->n_node, fs);
    }
    launch_field_advance_batch(b->d_field, b->node_items, b->n_node, b->j_filter == 0, true, b->tile, b->halo,
                               fs);
    if (fork) (void)hipEventRecord(b->ev_join, b->side);
    SortBatch sb;
    sb.descs = b->d_sort;
    sb.count_items = b->count_items;
    sb.n_count = b->n_count;
    sb.scan_items = b->scan_items;
    sb.n_scan = b->n_scan;
    sb.plan_items = b->plan_items;
    sb.n_plan = b->n_plan;
    sb.max_blocks = b->max_blocks;
    if (sort) launch_sort_batch(sb, (b->sims[0]->cfg.flags & PIC_FLAG_MOTION_SORT) != 0, stream);
    if (fork) (void)hipStreamWaitEvent(stream, b->ev_join, 0);
}

}  // namespace

extern "C" {

int pic_batch_query(int n, const pic_config *cfgs, size_t *bytes)
{
    if (!bytes) return PIC_EINVAL;
    const int rc = batch_validate(n, cfgs);
    if (rc) return rc;
    *bytes = batch_layout(n, cfgs).total;
    return PIC_OK;
}

int pic_batch_init(int n, const pic_config *cfgs, const pic_buffers *bufs, void *batch_work, size_t batch_bytes,
                   hipStream_t stream, pic_batch **out)
{
    if (!out || !bufs) return PIC_EINVAL;
    *out = nullptr;
    int rc = batch_validate(n, cfgs);
    if (rc) return rc;
    const BatchLayout L = batch_layout(n, cfgs);
    if (!batch_work || batch_bytes < L.total || ((uintptr_t)batch_work) % kAlign) return PIC_EINVAL;

    pic_batch *B = new (std::nothrow) pic_batch();
    if (!B) return PIC_EINVAL;
    rc = hip_ok(hipStreamCreateWithFlags(&B->side, hipStreamNonBlocking));
    if (rc == PIC_OK) rc = hip_ok(hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming));
    if (rc == PIC_OK) rc = hip_ok(hipEventCreateWithFlags(&B->ev_join, hipEventDisableTiming));
    if (rc) {
        pic_batch_destroy(B);
        return rc;
    }
    for (int i = 0; i < n; ++i) {
        pic_sim *S = nullptr;
        rc = init_sim(&cfgs[i], &bufs[i], stream, &S, false);
        if (rc) {
            pic_batch_destroy(B);
            return rc;
        }
        B->sims.push_back(S);
    }
    B->tile = cfgs[0].tile;
    B->j_filter = cfgs[0].j_filter;
    B->jm = j_mode(&cfgs[0]);
    B->dm = d_mode(&cfgs[0]);
    B->replicas = cfgs[0].j_replicas ? cfgs[0].j_replicas : default_replicas(&cfgs[0]);
    B->cadence = cadence_of(&cfgs[0]);
    B->halo = halo_of(&cfgs[0]);
    B->ppl = ppl_of(&cfgs[0]);
    B->phase = 0;
    char *d = (char *)batch_work;
    B->dev = d;
    B->d_push = (PushArgs *)(d + L.d_push);
    B->d_jr = (JReduceArgs *)(d + L.d_jr);
    B->d_sort = (SortArgs *)(d + L.d_sort);
    B->d_field = (FieldArgs *)(d + L.d_field);
    B->d_filter = (FilterArgs *)(d + L.d_filter);
    B->push_items = (int4 *)(d + L.push_items);
    B->node_items = (int4 *)(d + L.node_items);
    B->count_items = (int4 *)(d + L.count_items);
    B->scan_items = (int4 *)(d + L.scan_items);
    B->plan_items = (int4 *)(d + L.plan_items);
    B->n_push = L.n_push;
    B->n_node = L.n_node;
    B->n_count = L.n_count;
    B->n_scan = L.n_scan;
    B->n_plan = L.n_plan;
    B->max_blocks = 0;
    for (int i = 0; i < n; ++i) {
        const int nt = (cfgs[i].nx / cfgs[i].tile) * (cfgs[i].ny / cfgs[i].tile);
        B->max_blocks = std::max(B->max_blocks, (nt + kScanBlock - 1) / kScanBlock);
    }

    // host images of the descriptors and work tables
    std::vector<PushArgs> hp(n);
    std::vector<JReduceArgs> hj(n);
    std::vector<SortArgs> hs(n);
    std::vector<FieldArgs> hf(n);
    std::vector<FilterArgs> hfl(2 * n);
    std::vector<int4> push_items, node_items, count_items, scan_items, plan_items;
    std::vector<std::pair<double, int>> cost(n);
    for (int i = 0; i < n; ++i) {
        const pic_sim *S = B->sims[i];
        hp[i] = push_args(S, true);
        hj[i] = jreduce_args(S);
        hs[i] = sort_args(S, !(S->cfg.flags & PIC_FLAG_MOTION_SORT));
        hf[i] = field_args(S, S->cfg.j_filter == 0, true);
        hfl[i] = filter_args(S, 0);
        hfl[n + i] = filter_args(S, 1);
        int64_t np = 0;
        for (int s = 0; s < S->cfg.n_species; ++s) np += S->cfg.species[s].n;
        cost[i] = {-(double)np / S->n_tiles, i};   // particles per tile, largest first
        for (int by = 0; by < (S->cfg.ny + 3) / 4; ++by)
            for (int bx = 0; bx < (S->cfg.nx + 63) / 64; ++bx) node_items.push_back(make_int4(i, bx, by, 0));
        for (int s = 0; s < S->cfg.n_species; ++s) {
            for (int k = 0; k < (S->n_tiles + kScanBlock - 1) / kScanBlock; ++k)
                count_items.push_back(make_int4(i, s, k, 0));
            scan_items.push_back(make_int4(i, s, 0, 0));
            for (int k = 0; k < (S->n_tiles + kSortWaves - 1) / kSortWaves; ++k)
                plan_items.push_back(make_int4(i, s, k, 0));
        }
    }
    std::sort(cost.begin(), cost.end());
    for (const auto &c : cost)
        for (int t = 0; t < B->sims[c.second]->n_tiles; ++t) push_items.push_back(make_int4(c.second, t, 0, 0));

    auto up = [&](void *dst, const void *src, size_t bytes) {
        if (rc == PIC_OK && bytes) rc = hip_ok(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream));
    };
    up(B->d_push, hp.data(), n * sizeof(PushArgs));
    up(B->d_jr, hj.data(), n * sizeof(JReduceArgs));
    up(B->d_sort, hs.data(), n * sizeof(SortArgs));
    up(B->d_field, hf.data(), n * sizeof(FieldArgs));
    up(B->d_filter, hfl.data(), 2 * n * sizeof(FilterArgs));
    up(B->push_items, push_items.data(), push_items.size() * sizeof(int4));
    up(B->node_items, node_items.data(), node_items.size() * sizeof(int4));
    up(B->count_items, count_items.data(), count_items.size() * sizeof(int4));
    up(B->scan_items, scan_items.data(), scan_items.size() * sizeof(int4));
    up(B->plan_items, plan_items.data(), plan_items.size() * sizeof(int4));
    if (rc == PIC_OK) rc = hip_ok(hipStreamSynchronize(stream));

    if (rc) {
        pic_batch_destroy(B);
        return rc;
    }
    *out = B;
    return PIC_OK;
}

int pic_batch_step(pic_batch *B, int nsteps, hipStream_t stream)
{
    if (!B || nsteps < 0) return PIC_EINVAL;
    int k = 0;
    while (k < nsteps) {
        if (B->exec && B->phase == 0 && nsteps - k >= B->cadence) {
            // one captured cadence cycle: cadence steps, the last with the sort
            if (hipGraphLaunch(B->exec, stream) != hipSuccess) return PIC_EHIP;
            k += B->cadence;
        } else {
            const bool sort = B->phase + 1 == B->cadence;
            batch_enqueue_step(B, sort, B->phase == 0, stream);
            B->phase = sort ? 0 : B->phase + 1;
            k += 1;
        }
    }
    // the members' own record of unsorted pushes (pic_batch_sim handles)
    for (pic_sim *S : B->sims) S->since_sort = B->phase;
    return hip_ok(hipGetLastError());
}

int pic_batch_capture(pic_batch *B, hipStream_t stream)
{
    if (!B || !stream) return PIC_EINVAL;
    if (B->exec) {
        (void)hipGraphExecDestroy(B->exec);
        B->exec = nullptr;
    }
    if (B->graph) {
        (void)hipGraphDestroy(B->graph);
        B->graph = nullptr;
    }
    if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return PIC_EHIP;
    for (int k = 0; k < B->cadence; ++k) batch_enqueue_step(B, k + 1 == B->cadence, k == 0, stream);
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(stream, &g) != hipSuccess || !g) return PIC_EHIP;
    B->graph = g;
    if (hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        B->exec = nullptr;
        return PIC_EHIP;
    }
    return PIC_OK;
}

pic_sim *pic_batch_sim(pic_batch *B, int i)
{
    if (!B || i < 0 || i >= (int)B->sims.size()) return nullptr;
    return B->sims[i];
}

int pic_batch_sync(pic_batch *B, hipStream_t stream)
{
    if (!B) return PIC_EINVAL;
    SortBatch sb;
    sb.descs = B->d_sort;
    sb.count_items = B->count_items;
    sb.n_count = B->n_count;
    sb.scan_items = B->scan_items;
    sb.n_scan = B->n_scan;
    sb.plan_items = B->plan_items;
    sb.n_plan = B->n_plan;
    sb.max_blocks = B->max_blocks;
    launch_fill_batch(sb, stream);   // members without a pending fill have zero fill counts
    launch_publish_batch(sb, B->phase == 0, stream);
    return hip_ok(hipGetLastError());
}

int pic_batch_check(pic_batch *B, hipStream_t stream)
{
    if (!B) return PIC_EINVAL;
    int first = PIC_OK;
    for (pic_sim *S : B->sims) {
        const int rc = read_errors(S, stream);
        if (rc && first == PIC_OK) first = rc;
    }
    return first;
}

void pic_batch_destroy(pic_batch *B)
{
    if (!B) return;
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    for (pic_sim *S : B->sims) pic_destroy(S);
    if (B->side) {
        (void)hipStreamSynchronize(B->side);
        (void)hipStreamDestroy(B->side);
    }
    if (B->ev_fork) (void)hipEventDestroy(B->ev_fork);
    if (B->ev_join) (void)hipEventDestroy(B->ev_join);
    delete B;
}

}  // extern "C"

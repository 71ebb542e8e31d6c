// Definitions the particle push kernel (k_push.hip) is compiled from,
// shared with the launchers and the sort: limits, the count record, device
// error bits, accumulation modes, the LDS budget, the particle and push
// argument structures and the wavefront split of a tile section.  Kept apart
// so that the push kernel's source is exactly k_push.hip and this file.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pic.h"

namespace pic {

// A pointer into device global memory, marked as such: loads and stores
// through it are global_* instructions (scalar base + 32-bit lane offset)
// rather than flat ones, which a kernel would otherwise issue for pointers it
// reads from memory (the batched kernels' per-simulation descriptors).
#define PIC_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ PIC_GLOBAL T *gp(T *p)
{
    return (PIC_GLOBAL T *)p;
}
__device__ __forceinline__ void set_err(int *err, int bits)
{
    __hip_atomic_fetch_or(gp(err), bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int kMaxSpecies = PIC_MAX_SPECIES;
constexpr int kBlock = 256;          // threads per sort / stencil block (4 wavefronts)
constexpr int kSortWaves = kBlock / 64;   // tiles per sort plan / scatter block (one per wavefront)
constexpr int kCntStride = 32;       // ints per tile in the count record
constexpr int kScanBlock = 256;      // tiles per block of the tile-count scan

// Wavefronts that push one tile (one workgroup of 64 * W threads): 4 up to
// 16 x 16 tiles; 8 for 32 x 32 tiles, whose 70 KB of LDS (E/B halo, current,
// motion queues) let two workgroups share a compute unit, so one tile's
// staging and write-out overlap the other's particle stream.
__host__ __device__ constexpr int push_waves(int T) { return T >= 32 ? 8 : 4; }
// LDS layout of the push kernel.  Up to 16 x 16 tiles, where LDS is plentiful:
// each E/B entry holds its cell and the next one in x (one 16-byte read per
// stencil row of two components), and leavers are buffered per wavefront and
// written out as whole lines.  32 x 32 tiles: one cell per entry and leaver
// copies straight from registers, which is what lets two workgroups share a CU.
__host__ __device__ constexpr bool push_packed(int T) { return T < 32; }
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
    kErrOverflow = 16, // a tile holds 2^31 particles or more (its fixed-point current could overflow)
    kErrGroup = 32,  // caller particles not grouped by tile (cells in range)
};

// Current accumulation modes of the push kernel.
enum : int {
    kJFixed = 0,   // exact int64 fixed point in LDS (default)
    kJFloat = 1,   // FP32 LDS atomics, compensated replica sum
};

// Fixed-point resolution: one current contribution of the largest possible
// magnitude (the particle charge of the largest species times a full cell of
// motion, or at the speed of light for Jz) is 2^30 units; each contribution
// is the FP32 product truncated to a unit, and the sums are exact.
constexpr float kFixedScale = 1073741824.0f;

// deposit scheme of the push kernel
constexpr int kDepVB = 0;          // Villasenor-Buneman with the 1/2/3-piece split (Eqs. 13-16)
constexpr int kDepEsirkepov = 1;   // Esirkepov's density decomposition (variant)
// The quadratic particle shape (B-spline of order two, three nodes per axis):
// the field gather at each component's staggered point and Esirkepov's
// current with that shape.  The shape reaches one node further than the
// linear one, so the push stages a halo one cell wider than the sort cadence
// alone needs.
constexpr int kDepQuad = 2;
// extra halo cells the deposit scheme's shape needs beyond the cadence's
__host__ __device__ constexpr int shape_pad(int DM) { return DM == kDepQuad ? 1 : 0; }

constexpr int kLdsBytes = 160 * 1024;   // LDS of one gfx950 compute unit
constexpr int kMotionBuf = 64;           // queued face-crossing motions per wavefront
constexpr int kLeaverBuf = 64;           // leavers buffered per wavefront (packed layout)
// one ballot can add a whole wavefront to either buffer
static_assert(kMotionBuf >= 64 && kLeaverBuf >= 64, "per-wavefront LDS buffers must hold 64 entries");

// Static LDS of the push kernel for tile T, R current replicas, mode JM and
// halo pad H (the sort cadence: between two sorts a particle may stray up to
// H - 1 cells outside its tile, so the E/B halo holds cells -H..T+H-1 and
// the current halo nodes -H..T+H).
constexpr int push_lds_bytes(int T, int R, int JM, int H = 1)
{
    return (T + 2 * H) * (T + 2 * H) * (push_packed(T) ? 48 : 24) +
           R * 3 * (T + 2 * H + 1) * (T + 2 * H + 1) * (JM == kJFixed ? 8 : 4) +
           kMaxSpecies * (9 + push_waves(T)) * 4 + push_waves(T) * 6 * kMotionBuf * 4 +
           (push_packed(T) ? push_waves(T) * 7 * kLeaverBuf * 4 : 0) + push_waves(T) * 64 * 4;
}

// Sort cadences the push kernel is built for: every 1, 2 or 4 steps, with
// the fixed-point current and one LDS copy of it when above 1.  A node's
// current halo then still overlaps at most one neighbour per axis (2H + 1 <=
// T), a position outside the tile has one periodic image within the pad
// (2H - 2 < T), and the LDS fits.
// Waves per SIMD a push kernel is compiled for (its register budget): the
// workgroups of its size that fit a CU's LDS, at most 4 waves per SIMD (128
// VGPRs).  A 4-wavefront workgroup (tiles up to 16 x 16) puts one wave on
// each SIMD, an 8-wavefront one (32 x 32) two.
constexpr int push_min_waves(int T, int R, int JM, int H)
{
    return T < 32 ? (kLdsBytes / push_lds_bytes(T, R, JM, H) < 4 ? kLdsBytes / push_lds_bytes(T, R, JM, H) : 4)
                  : (2 * push_lds_bytes(T, R, JM, H) <= kLdsBytes ? 4 : 2);
}

constexpr bool cadence_ok(int T, int H)
{
    return (H == 1 || H == 2 || H == 4) && 2 * H + 1 <= T && push_lds_bytes(T, 1, kJFixed, H) <= kLdsBytes;
}

// The cell of a particle as the push and the sort stream it: 16 bits, the
// cell's offset (lx, ly) from the first cell of the tile whose section holds
// the particle, each a signed byte, lx | ly << 8.  Inside the tile both lie
// in [0, tile); a particle that has left it is up to a few cells outside,
// across the periodic seam too (no wrap: the offset says which neighbour it
// went to).  The sort copies the particles it moves with their cells
// relative to their new tile, but one that entered a tile and already sits
// in that tile's new section stays where it is, its cell still relative to
// the tile it came from: so in a sorted state (no push since the last sort)
// a cell is relative to its tile modulo the tile edge, and every reader
// then takes it modulo the edge.  The caller's arrays keep the whole-grid
// cell ix | iy << 16, written from these when the caller is to read them.
__host__ __device__ __forceinline__ int tcell_pack(int lx, int ly) { return (lx & 0xff) | ((ly & 0xff) << 8); }
__device__ __forceinline__ int tcell_x(int c) { return __builtin_amdgcn_sbfe(c, 0, 8); }
__device__ __forceinline__ int tcell_y(int c) { return __builtin_amdgcn_sbfe(c, 8, 8); }
// a particle that left the moving window: (-128, -128), no tile
constexpr int kTCellRemoved = 0x8080;

// One species' particles as the kernels stream them: a structure of arrays
// (n entries each), tile-relative cells.
struct Parts {
    int16_t *cell;
    float *x, *y, *ux, *uy, *uz;
};

// The same with whole-grid cells ix | iy << 16 (the caller's arrays).
struct GParts {
    int32_t *cell;
    float *x, *y, *ux, *uy, *uz;
};

// One leaver's new particle data, written by the push and read by the sort:
// one aligned 32-byte record, so each copy is one memory sector on both sides
// (six separate arrays would cost six scattered sectors per leaver).
struct __attribute__((aligned(32))) LeaverRec {
    int32_t cell;
    float x, y, ux, uy, uz;
    int32_t pad[2];
};

// plain clang vectors (HIP's vector classes have no address-space-qualified
// assignment)
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef float vf2 __attribute__((ext_vector_type(2)));

// Write one leaver record as two vector stores (16 + 8 bytes).
__device__ __forceinline__ void put_leaver(LeaverRec *r, int64_t q, int cell, float x, float y, float ux, float uy,
                                           float uz)
{
    PIC_GLOBAL vf4 *d = (PIC_GLOBAL vf4 *)(r + q);
    d[0] = vf4{__int_as_float(cell), x, y, ux};
    *(PIC_GLOBAL vf2 *)(d + 1) = vf2{uy, uz};
}

struct SpeciesDev {
    int16_t *cell;        // tile-relative cells (tcell_pack)
    float *x, *y, *ux, *uy, *uz;
    const int32_t *off;   // tile_offset at the start of the step (n_tiles + 1)
    int32_t *cnt;         // [n_tiles][kCntStride]
    uint32_t *leav;       // [n]: leaver sub-lists, (slot - off[t]) << 4 | direction
    LeaverRec *lrec;      // [n]: the leavers' new particle data, same positions as leav
    // a fill left by the last sort: tile t's fcount[t] holes, slots fhole[off[t] + r]
    // ascending, take the staged particles fsrc[off[t] + r]; wavefront w's first
    // is rank fbase[t W + w].  The push zeroes fcount[t].
    int32_t *fcount;
    const int32_t *fbase;
    const int32_t *fhole;
    const LeaverRec *fsrc;
    // the motion-class sort's staging arrays (read instead of the above when
    // PushArgs::stg_live is set), or null
    const int16_t *scell;
    const float *sx, *sy, *sux, *suy, *suz;
    int32_t n;
    float h;              // (q/m) dt / 2
    float fq;             // charge in accumulator units: q / max|q| (x kFixedScale in fixed mode)
};

struct PushArgs {
    const float *fld;     // Ex Ey Ez Bx By Bz planes
    float *bh;            // or null: B after the first half step of the field advance (three planes,
                          // each tile writes its cells from its staged halo)
    float hdx, hdy;       // (dt/2)/dx, (dt/2)/dy
    float *jtile;         // [n_tiles][3][(T+2H+1)^2], physical current of each tile halo
    int *err;
    int nx, ny, ntx, nty;
    float cx, cy;         // dt/dx, dt/dy
    float ju[3];          // accumulator unit -> physical Jx, Jy, Jz
    int n_species;
    int rebase;           // the push follows a sort: each cell is relative to the tile modulo its edge
    const int *stg_live;  // nonzero: the particles wait in the motion-class sort's staging arrays
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

struct JReduceArgs {
    const float *jtile;
    float *J;             // the Jx plane; Jy, Jz follow
    int nx, ny, ntx, nty;
};

}  // namespace pic

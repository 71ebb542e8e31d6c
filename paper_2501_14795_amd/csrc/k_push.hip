// Particle push + current deposit for one tile per workgroup, and the fold of
// the per-tile current halos into the global J planes.
//
// Per tile (Sec. 4.2.2 maps one tile to one work-group; redesigned here for
// gfx950 wave64 + LDS):
//   1. stage the tile's E/B halo (cells -H..T+H-1 on each axis; H = 1 when
//      particles are sorted every step, H = k when every k steps, as a
//      particle then strays up to k - 1 cells outside its tile) in LDS, the
//      two components interpolated at the same points side by side, so the
//      two x-neighbours of a stencil row come in one ds_read2;
//   2. the 64-aligned particle chunks covering the tile's section are split
//      into contiguous runs, one per wavefront (4 wavefronts per tile up to
//      16 x 16 tiles, 8 for 32 x 32 tiles, two such workgroups per CU); every chunk is one
//      coalesced buffer load per SoA array (per-tile buffer base in SGPRs):
//      the cell as 16 bits relative to the tile, x, y, ux, uy, uz as FP32
//      (22 bytes a particle), and there is no block barrier in the loop; the
//      holes the last sort left get their particles from its staging records
//      as the chunk is loaded, and after a motion-class sort the chunks come
//      from its staging arrays;
//   3. per particle: bilinear interpolation at the staggered points
//      (Sec. 3.1), Boris push (Eqs. 6-10), move (Eq. 11), and the
//      Villasenor-Buneman current (Eqs. 13-16) of each of the 1, 2 or 3 pieces
//      of the motion (Figs. 3.4-3.5), added into the LDS current of the tile.
//      A motion that stays in its cell (~85% of them) is one piece, deposited
//      at once; one that crosses a cell face goes whole to a per-wavefront LDS
//      queue, drained 64 motions at a time, where it is cut into its pieces --
//      so the cutting and the extra deposits run on full wavefronts instead of
//      on the few lanes of each wavefront that cross:
//      With the quadratic shape (kDepQuad) the gather weights three points
//      per axis and the current is Esirkepov's with that shape: a motion
//      whose nearest node stays the same is deposited at once on 3 x 3
//      nodes, one whose nearest node changes goes to the queue and to 4 x 4.
//        kJFixed  exact int64 fixed point (ds_add_u64): every contribution is
//                 the FP32 product truncated to 2^-30 of the largest
//                 possible contribution, the sums are exact, so J does not
//                 depend on the order of the additions -- bit-reproducible;
//        kJFloat  FP32 ds_add_f32 into one of R replicas (lane mod R), the
//                 replicas summed with compensation at the end.  Kept as the
//                 reference mode: on gfx950 FP32 LDS atomics are several times
//                 slower than integer ones;
//   4. particles whose tile changed are appended, in slot order, to the
//      wavefront's leaver sub-list (ballot + mbcnt) with a copy of their new
//      data, and counted per direction -- the input of the strict sort
//      (Sec. 4.3, step 1);
//   5. the tile's (T+2H+1)^2 current halo is converted to physical units and
//      written out; k_j_reduce (or the E step of the field advance) then adds
//      the up-to-four overlapping tile halos of every node in a fixed order
//      with compensation (no global atomics); in pic_step the tile also writes
//      the first B half step of its own cells from its staged E/B halo.
#include <type_traits>

#include "pic_internal.h"
#include "pic_fold.h"
#include "pic_yee.h"

namespace pic {

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ float lerpf(float a, float b, float w) { return fmaf(w, b - a, a); }

__device__ __forceinline__ float clamp01(float v) { return fminf(fmaxf(v, 0.0f), 1.0f); }

__device__ __forceinline__ int lane_rank(unsigned long long m)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

constexpr int kRsrcWord3 = 0x00020000;   // raw 32-bit buffer access, gfx9 family

struct Stream6 {
    __amdgpu_buffer_rsrc_t cell, x, y, ux, uy, uz;
};


__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *base, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, bytes, kRsrcWord3);
}

// Views of six particle arrays from slot `base`, `bytes` bytes of the 32-bit ones.
__device__ __forceinline__ Stream6 stream6(const int16_t *cell, const float *x, const float *y, const float *ux,
                                           const float *uy, const float *uz, int base, int bytes)
{
    Stream6 s;
    s.cell = rsrc(cell + base, bytes / 2);
    s.x = rsrc(x + base, bytes);
    s.y = rsrc(y + base, bytes);
    s.ux = rsrc(ux + base, bytes);
    s.uy = rsrc(uy + base, bytes);
    s.uz = rsrc(uz + base, bytes);
    return s;
}

// Cache policy of the particle stream's buffer loads and stores: the
// non-temporal hint (the nt bit of gfx950's cache-policy operand).  Every
// particle is read and written once per step, so keeping the stream out of
// the L2 and the Infinity Cache leaves them to what is reused -- the E/B and
// current halos, the leaver lists, and the fields, tile halos and lists the
// j_reduce, sort and field kernels of the same step read (measured: push
// -12 %, the rest of the step -20 %; either hint alone gains little).
constexpr int kLoadCpol = 2;
constexpr int kStoreCpol = 2;

__device__ __forceinline__ float ldf(__amdgpu_buffer_rsrc_t r, int off)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, kLoadCpol));
}

__device__ __forceinline__ void stf(__amdgpu_buffer_rsrc_t r, int off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, 0, kStoreCpol);
}

// LDS current accumulator of one mode.
template <int JM>
struct JAcc;

// Exact fixed point.  A contribution a*w (|a*w| <= 2^30 units: the largest
// particle charge moving one cell, or at c for Jz) is rounded once, in the
// FP32 product, then truncated to a whole unit (2^-30 of the largest
// contribution) and added as a signed 64-bit integer.  The sums are exact,
// so J does not depend on the order of the additions; they cannot overflow
// while a tile holds fewer than 2^31 particles (checked), since a particle
// adds to one node at most three times per component.
template <>
struct JAcc<kJFixed> {
    using T = unsigned long long;   // two's complement int64 (ds_add_u64)
    __device__ static __forceinline__ void add(T *p, float a, float w)
    {
        const int v = (int)(a * w);
        atomicAdd(p, (T)(long long)v);
    }
    // int64 -> float without FP64: s = hi 2^32 + lo with lo a signed 32-bit
    // remainder, so a small negative sum is not the difference of two large
    // numbers; hi is exact in FP32 while |s| < 2^55
    __device__ static __forceinline__ float value(const T *p, int replicas, int stride, float unit, int *)
    {
        long long s = 0;
        for (int r = 0; r < replicas; ++r) s += (long long)p[r * stride];
        const int hi = (int)((s + 0x80000000ll) >> 32);
        const int lo = (int)(s - ((long long)hi << 32));
        return fmaf((float)hi, 4294967296.0f, (float)lo) * unit;
    }
};

template <>
struct JAcc<kJFloat> {
    using T = float;
    __device__ static __forceinline__ void add(T *p, float a, float w) { atomicAdd(p, a * w); }
    __device__ static __forceinline__ float value(const T *p, int replicas, int stride, float unit, int *)
    {
        // compensated (TwoSum) sum of the replicas
        float s = 0.0f, c = 0.0f;
        for (int r = 0; r < replicas; ++r) {
            const float v = p[r * stride];
            const float t = s + v;
            const float bp = t - s;
            c += (s - (t - bp)) + (v - bp);
            s = t;
        }
        return (s + c) * unit;
    }
};

// LDS index of tile-relative node (cx, cy) in the (T+2H+1)^2 current halo
// (nodes -H..T+H per axis).
template <int NJ, int H>
__device__ __forceinline__ int jcell(int cx, int cy)
{
    return __mul24(cy + H, NJ) + (cx + H);   // 24-bit multiply: full rate
}

// Current of one piece of the motion inside the cell at halo index b, from
// (xa, ya) in that cell's frame by (dxk, dyk), in accumulator units (fq =
// particle charge in those units; az = fq vz times the piece's share of the
// step).  Jx/Jy: the Villasenor-Buneman face fluxes; Jz: az times the exact
// time average of each corner's bilinear weight, w_mid +- dxk dyk / 12.
// The piece is given by its displacement, not its end point: for a small
// motion the difference of two offsets near 1/2 would carry an absolute
// rounding error of half an ulp of the offset (3e-8), a large relative
// error of the flux when the motion is a thousandth of a cell.
template <int NJ, int JM>
__device__ __forceinline__ void deposit_piece(typename JAcc<JM>::T *sj, int b, float xa, float ya, float dxk,
                                              float dyk, float az, float fq)
{
    constexpr int P = NJ * NJ;
    using A = JAcc<JM>;
    const float xm = fmaf(0.5f, dxk, xa), ym = fmaf(0.5f, dyk, ya);
    const float ax = fq * dxk, ay = fq * dyk;
    const float c = dxk * dyk * (1.0f / 12.0f);
    const float xm1 = 1.0f - xm, ym1 = 1.0f - ym;
    A::add(&sj[b], ax, ym1);
    A::add(&sj[b + NJ], ax, ym);
    A::add(&sj[P + b], ay, xm1);
    A::add(&sj[P + b + 1], ay, xm);
    A::add(&sj[2 * P + b], az, fmaf(xm1, ym1, c));
    A::add(&sj[2 * P + b + 1], az, fmaf(xm, ym1, -c));
    A::add(&sj[2 * P + b + NJ], az, fmaf(xm1, ym, -c));
    A::add(&sj[2 * P + b + NJ + 1], az, fmaf(xm, ym, c));
}

// Villasenor-Buneman current of a motion that crosses one or two cell faces,
// from (x, y) in the cell at halo index b by (dX, dY) cells (|dX|, |dY| < 1):
// the motion is cut at the face crossings in time order, and piece k lies in
// the cell reached after k crossings, in whose frame it starts (az: fq vz
// for the whole step, shared among the pieces by duration).  The pieces'
// displacements are differences of the motion's cumulative displacement at
// the crossings -- the distance to the face on the crossing axis (exact),
// the crossing time times the motion on the other -- so they add up to
// (dX, dY) to within an ulp of the motion.
template <int NJ, int JM>
__device__ __forceinline__ void deposit_split(typename JAcc<JM>::T *sj, int b, float x, float y, float dX,
                                              float dY, float az, float fq)
{
    const float x1 = x + dX, y1 = y + dY;
    const int sxn = x1 >= 1.0f ? 1 : (x1 < 0.0f ? -1 : 0);
    const int syn = y1 >= 1.0f ? 1 : (y1 < 0.0f ? -1 : 0);
    const float ex = sxn > 0 ? 1.0f : 0.0f;   // x face crossed (start-cell frame)
    const float ey = syn > 0 ? 1.0f : 0.0f;
    const float tcx = sxn ? clamp01((ex - x) * __builtin_amdgcn_rcpf(dX)) : 1.0f;
    const float tcy = syn ? clamp01((ey - y) * __builtin_amdgcn_rcpf(dY)) : 1.0f;
    const bool xfirst = sxn != 0 && (syn == 0 || tcx <= tcy);
    const bool three = sxn != 0 && syn != 0;
    const float t1 = xfirst ? tcx : tcy;
    const float t2 = xfirst ? tcy : tcx;
    // cumulative displacement at the first and second crossing
    const float X1 = xfirst ? ex - x : t1 * dX, Y1 = xfirst ? t1 * dY : ey - y;
    const float X2 = three ? (xfirst ? t2 * dX : ex - x) : dX;
    const float Y2 = three ? (xfirst ? ey - y : t2 * dY) : dY;
    // piece 0, in the start cell
    deposit_piece<NJ, JM>(sj, b, x, y, X1, Y1, az * t1, fq);
    // piece 1, after the first crossing
    const int ox = xfirst ? sxn : 0, oy = xfirst ? 0 : syn;
    deposit_piece<NJ, JM>(sj, b + oy * NJ + ox, clamp01(x + X1 - (float)ox), clamp01(y + Y1 - (float)oy), X2 - X1,
                          Y2 - Y1, az * ((three ? t2 : 1.0f) - t1), fq);
    // piece 2, after both crossings
    if (three)
        deposit_piece<NJ, JM>(sj, b + syn * NJ + sxn, clamp01(x + X2 - (float)sxn), clamp01(y + Y2 - (float)syn),
                              dX - X2, dY - Y2, az * (1.0f - t2), fq);
}

// Esirkepov's current of a whole straight motion (the variant deposit) from
// (x, y) in the cell at halo index b to (x1, y1) in that cell's frame
// (x1, y1 in (-1, 2)), on the 4 x 4 nodes around it.  Node weights of the
// linear shape before (S0) and after (S1), DS = S1 - S0:
//   W^x_kl = DSx_k (S0y_l + DSy_l / 2)   -> Jx at (k+1/2, l) = -sum_{k'<=k} W^x
//   W^y_kl = DSy_l (S0x_k + DSx_k / 2)   -> Jy likewise
//   W^z_kl = S0x S0y + (DSx S0y + S0x DSy) / 2 + DSx DSy / 3
// in accumulator units (fq: particle charge; az: fq vz for the whole step).
// Within one cell it equals the Villasenor-Buneman piece.
template <int NJ, int JM>
__device__ __forceinline__ void deposit_esirkepov(typename JAcc<JM>::T *sj, int b, float x, float y, float x1,
                                                  float y1, float az, float fq)
{
    constexpr int P = NJ * NJ;
    using A = JAcc<JM>;
    const float s0x[4] = {0.0f, 1.0f - x, x, 0.0f}, s0y[4] = {0.0f, 1.0f - y, y, 0.0f};
    float dsx[4], dsy[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        dsx[k] = fmaxf(0.0f, 1.0f - fabsf(x1 - (float)(k - 1))) - s0x[k];
        dsy[k] = fmaxf(0.0f, 1.0f - fabsf(y1 - (float)(k - 1))) - s0y[k];
    }
    const int o = b - NJ - 1;   // node (-1, -1) relative to the cell
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        const float gy = fmaf(0.5f, dsy[l], s0y[l]);
        float run = 0.0f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            run = fmaf(-dsx[k], gy, run);
            A::add(&sj[o + l * NJ + k], fq, run);
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float gx = fmaf(0.5f, dsx[k], s0x[k]);
        float run = 0.0f;
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            run = fmaf(-dsy[l], gx, run);
            A::add(&sj[P + o + l * NJ + k], fq, run);
        }
    }
#pragma unroll
    for (int l = 0; l < 4; ++l)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float w = s0x[k] * s0y[l] + 0.5f * (dsx[k] * s0y[l] + s0x[k] * dsy[l]) +
                            dsx[k] * dsy[l] * (1.0f / 3.0f);
            A::add(&sj[2 * P + o + l * NJ + k], az, w);
        }
}

// Quadratic B-spline weights of the three nodes around a position e in
// [-1/2, 1/2) from the middle one: at distances 1 + e, e, 1 - e.
__device__ __forceinline__ void quad_w3(float e, float &wm, float &w0, float &wp)
{
    const float a = 0.5f - e, b = 0.5f + e;
    wm = 0.5f * a * a;
    w0 = fmaf(-e, e, 0.75f);
    wp = 0.5f * b * b;
}

// Quadratic B-spline weight of a node at distance d (cells).
__device__ __forceinline__ float quad_w(float d)
{
    const float a = fabsf(d), b = 1.5f - a;
    return a <= 0.5f ? fmaf(-a, a, 0.75f) : (a < 1.5f ? 0.5f * b * b : 0.0f);
}

// Esirkepov's current with the quadratic shape (kDepQuad) of a whole straight
// motion from (x, y) in the cell at halo index b by (dX, dY) cells.  The
// shape covers the three nodes nearest the particle; the nearest node moves
// by at most one, so the four nodes from one below the lower of the two
// nearest nodes hold the shape before and after (per axis the window starts
// 0, 1 or 2 nodes below the cell).  With the window's node weights S0, S1
// and DS = S1 - S0, the same decomposition as deposit_esirkepov:
//   W^x_kl = DSx_k (S0y_l + DSy_l / 2) -> Jx at (k+1/2, l) = -sum_{k'<=k} W^x
//   W^y likewise, W^z_kl = S0x S0y + (DSx S0y + S0x DSy) / 2 + DSx DSy / 3,
// each in accumulator units (|run| <= 3/4, W^z <= 9/16: within the
// fixed-point range of one contribution).
template <int NJ, int JM>
__device__ __forceinline__ void deposit_quad(typename JAcc<JM>::T *sj, int b, float x, float y, float dX, float dY,
                                             float az, float fq)
{
    constexpr int P = NJ * NJ;
    using A = JAcc<JM>;
    const float x1 = x + dX, y1 = y + dY;
    // window start relative to the cell: min(nearest before, nearest after) - 1
    const int nx0 = x >= 0.5f ? 1 : 0, ny0 = y >= 0.5f ? 1 : 0;
    // x1, y1 lie in (-1, 2) (|dX|, |dY| < 1): their nearest node -1 .. 2 (the
    // clamp keeps the window inside the halo whatever the input)
    const int nx1 = min(max((int)floorf(x1 + 0.5f), -1), 2), ny1 = min(max((int)floorf(y1 + 0.5f), -1), 2);
    const int wx = min(nx0, nx1) - 1, wy = min(ny0, ny1) - 1;
    float s0x[4], s0y[4], dsx[4], dsy[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float px = (float)(wx + k), py = (float)(wy + k);
        s0x[k] = quad_w(x - px);
        dsx[k] = quad_w(x1 - px) - s0x[k];
        s0y[k] = quad_w(y - py);
        dsy[k] = quad_w(y1 - py) - s0y[k];
    }
    const int o = b + wy * NJ + wx;   // window node (0, 0)
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        const float gy = fmaf(0.5f, dsy[l], s0y[l]);
        float run = 0.0f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            run = fmaf(-dsx[k], gy, run);
            A::add(&sj[o + l * NJ + k], fq, run);
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float gx = fmaf(0.5f, dsx[k], s0x[k]);
        float run = 0.0f;
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            run = fmaf(-dsy[l], gx, run);
            A::add(&sj[P + o + l * NJ + k], fq, run);
        }
    }
#pragma unroll
    for (int l = 0; l < 4; ++l)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float w = s0x[k] * s0y[l] + 0.5f * (dsx[k] * s0y[l] + s0x[k] * dsy[l]) +
                            dsx[k] * dsy[l] * (1.0f / 3.0f);
            A::add(&sj[2 * P + o + l * NJ + k], az, w);
        }
}

// deposit_quad for a motion whose nearest node stays the same on both axes
// (the common case): the shape covers the same three nodes before and after,
// so a window of three per axis is exact -- 6 + 6 + 9 contributions instead
// of 12 + 12 + 16 (those of the fourth node are zero to rounding).  hx, hy:
// the nearest node relative to the cell (0 or 1).
template <int NJ, int JM>
__device__ __forceinline__ void deposit_quad3(typename JAcc<JM>::T *sj, int b, int hx, int hy, float x, float y,
                                              float dX, float dY, float az, float fq)
{
    constexpr int P = NJ * NJ;
    using A = JAcc<JM>;
    const float ex = x - (float)hx, ey = y - (float)hy;   // offsets from the nearest node, [-1/2, 1/2)
    float s0x[3], s0y[3], s1x[3], s1y[3], dsx[3], dsy[3];
    quad_w3(ex, s0x[0], s0x[1], s0x[2]);
    quad_w3(ey, s0y[0], s0y[1], s0y[2]);
    quad_w3(ex + dX, s1x[0], s1x[1], s1x[2]);
    quad_w3(ey + dY, s1y[0], s1y[1], s1y[2]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        dsx[k] = s1x[k] - s0x[k];
        dsy[k] = s1y[k] - s0y[k];
    }
    const int o = b + (hy - 1) * NJ + (hx - 1);   // window node (0, 0)
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const float gy = fmaf(0.5f, dsy[l], s0y[l]);
        float run = 0.0f;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            run = fmaf(-dsx[k], gy, run);
            A::add(&sj[o + l * NJ + k], fq, run);
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float gx = fmaf(0.5f, dsx[k], s0x[k]);
        float run = 0.0f;
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            run = fmaf(-dsy[l], gx, run);
            A::add(&sj[P + o + l * NJ + k], fq, run);
        }
    }
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float w = s0x[k] * s0y[l] + 0.5f * (dsx[k] * s0y[l] + s0x[k] * dsy[l]) +
                            dsx[k] * dsy[l] * (1.0f / 3.0f);
            A::add(&sj[2 * P + o + l * NJ + k], az, w);
        }
}

// The wavefront's queue of face-crossing motions: kMotionBuf entries of
// (halo index of the start cell, x, y, dX, dY, fq vz).

template <int NJ, int JM, int DM>
__device__ __forceinline__ void drain_motions(typename JAcc<JM>::T *sj, uint32_t (*pq)[kMotionBuf], int n,
                                              float fq, int lane)
{
    __builtin_amdgcn_wave_barrier();
    if (lane < n) {
        const int b = (int)pq[0][lane];
        const float x = __uint_as_float(pq[1][lane]), y = __uint_as_float(pq[2][lane]);
        const float dX = __uint_as_float(pq[3][lane]), dY = __uint_as_float(pq[4][lane]);
        const float az = __uint_as_float(pq[5][lane]);
        if constexpr (DM == kDepQuad)
            deposit_quad<NJ, JM>(sj, b, x, y, dX, dY, az, fq);
        else if constexpr (DM == kDepEsirkepov)
            deposit_esirkepov<NJ, JM>(sj, b, x, y, x + dX, y + dY, az, fq);
        else
            deposit_split<NJ, JM>(sj, b, x, y, dX, dY, az, fq);
    }
    __builtin_amdgcn_wave_barrier();
}

// Append the motions of the lanes with `has` set to the queue (slot order by
// lane), draining it first if they do not fit.  n: queue fill, uniform.
template <int NJ, int JM, int DM>
__device__ __forceinline__ void queue_motion(typename JAcc<JM>::T *sj, uint32_t (*pq)[kMotionBuf], int &n, bool has,
                                             int b, float x, float y, float dX, float dY, float az, float fq,
                                             int lane)
{
    const unsigned long long m = __ballot(has);
    const int c = __popcll(m);
    if (c == 0) return;
    if (n + c > kMotionBuf) {
        drain_motions<NJ, JM, DM>(sj, pq, n, fq, lane);
        n = 0;
    }
    if (has) {
        const int r = n + lane_rank(m);
        pq[0][r] = (uint32_t)b;
        pq[1][r] = __float_as_uint(x);
        pq[2][r] = __float_as_uint(y);
        pq[3][r] = __float_as_uint(dX);
        pq[4][r] = __float_as_uint(dY);
        pq[5][r] = __float_as_uint(az);
    }
    n += c;
}

// Write the n leavers buffered in LDS by one wavefront to the leaver list
// and the leaver copies, from position pos on (contiguous: whole lines).
__device__ __forceinline__ void flush_leavers(const SpeciesDev &sp, uint32_t (*lb)[kLeaverBuf], int n,
                                              int64_t pos, int lane)
{
    __builtin_amdgcn_wave_barrier();
    if (lane < n) {
        const int64_t q = pos + lane;
        gp(sp.leav)[q] = lb[0][lane];
        put_leaver(sp.lrec, q, (int)lb[1][lane], __uint_as_float(lb[2][lane]), __uint_as_float(lb[3][lane]),
                   __uint_as_float(lb[4][lane]), __uint_as_float(lb[5][lane]), __uint_as_float(lb[6][lane]));
    }
    __builtin_amdgcn_wave_barrier();
}

// One lane's particle of one chunk, as loaded (cell: tile-relative, tcell_pack).
struct Chunk {
    int cell;
    float x, y, ux, uy, uz;
};

// off: the byte offset of the slot in the 32-bit arrays (half of it in the
// 16-bit cell array)
__device__ __forceinline__ Chunk load_chunk(const Stream6 &st, int off)
{
    Chunk c;
    c.cell = (int)__builtin_amdgcn_raw_buffer_load_b16(st.cell, off >> 1, 0, kLoadCpol);
    c.x = ldf(st.x, off);
    c.y = ldf(st.y, off);
    c.ux = ldf(st.ux, off);
    c.uy = ldf(st.uy, off);
    c.uz = ldf(st.uz, off);
    return c;
}

// What a particle's step produces: its new state, its motion for the
// current, and where it goes.
struct Moved {
    bool valid, cross;   // in the wavefront's run; motion crosses a cell face
    int b;               // current-halo index of the start cell
    int ncell, dir;      // new whole-grid cell; direction of the new tile (4: same tile)
    int nlc;             // new tile-relative cell (the same tile's frame)
    int err;             // error bits (kErrOrder, kErrRange), valid lanes only
    float x, y, dX, dY, fqvz;
    float xn, yn, ux, uy, uz;
};

// Interpolation, Boris push and move of one particle (no side effects, no
// branches).  Lanes outside the run compute on a cell clamped into the halo,
// so their LDS reads stay in bounds; their results are discarded.
template <int T, int NJ, int NE, int H, int DM, class V2, class V1>
__device__ __forceinline__ Moved advance(const PushArgs &a, const Chunk &p, bool valid, bool rebase, int gx0,
                                         int gy0, bool tx_wrap, bool ty_wrap, float h, float fq, const V2 *s_exby,
                                         const V2 *s_eybx, const V1 *s_ez, const V1 *s_bz)
{
    Moved m;
    m.valid = valid;
    m.err = 0;
    const float x = p.x, y = p.y;
    // The cell relative to the tile.  Since the last sort the particle may
    // have left the tile by up to H - 1 cells.  Right after a sort (rebase)
    // it is inside the tile, and its cell is relative to the tile it was in
    // before the sort, up to H cells off: modulo T it is its cell here.
    // Anything further is flagged.
    // (The halo pad H is the sort cadence plus the shape's pad Q.)
    constexpr int Q = shape_pad(DM);
    int lx = tcell_x(p.cell), ly = tcell_y(p.cell);
    const int bl = rebase ? H - Q : H - 1 - Q;   // the band of cells allowed: -bl .. T - 1 + bl
    if (valid && ((unsigned)(lx + bl) >= (unsigned)(T + 2 * bl) || (unsigned)(ly + bl) >= (unsigned)(T + 2 * bl)))
        m.err |= kErrOrder;
    if (rebase) {
        lx &= T - 1;
        ly &= T - 1;
    }
    lx = min(max(lx, 1 - H + Q), T + H - 2 - Q);
    ly = min(max(ly, 1 - H + Q), T + H - 2 - Q);

    float Ex, By, Ey, Bx, Ez, Bz;
    if constexpr (DM == kDepQuad) {
        // ---- interpolation with the quadratic shape: per axis the three
        // sample points nearest the particle.  Points at whole cells: the
        // nearest is the cell's own or the next one (x >= 1/2), at offset
        // ex = x or x - 1; points at half cells: the nearest is the cell's,
        // at offset x - 1/2.  Stencil columns from ci / ch, rows from ri / rh
        // (LDS indices; within 1 .. NE - 1 by the clamp above).
        const int hx = x >= 0.5f ? 1 : 0, hy = y >= 0.5f ? 1 : 0;
        float ix3[3], hx3[3], iy3[3], hy3[3];
        quad_w3(x - (float)hx, ix3[0], ix3[1], ix3[2]);
        quad_w3(x - 0.5f, hx3[0], hx3[1], hx3[2]);
        quad_w3(y - (float)hy, iy3[0], iy3[1], iy3[2]);
        quad_w3(y - 0.5f, hy3[0], hy3[1], hy3[2]);
        const int ci = lx + hx - 1 + H, ch = lx - 1 + H;
        const int ri = ly + hy - 1 + H, rh = ly - 1 + H;
        Ex = By = Ey = Bx = Ez = Bz = 0.0f;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const int ei = __mul24(ri + r, NE), eh = __mul24(rh + r, NE);
            // the three values of a row: packed entries hold a cell and the next
            float2 p3[3], q3[3];
            float z3[3], b3[3];
            if constexpr (std::is_same<V2, float4>::value) {
                const float4 pa = s_exby[ei + ch], pb = s_exby[ei + ch + 2];
                const float4 qa = s_eybx[eh + ci], qb = s_eybx[eh + ci + 2];
                const float2 za = s_ez[ei + ci], zb = s_ez[ei + ci + 2];
                const float2 ba = s_bz[eh + ch], bb = s_bz[eh + ch + 2];
                p3[0] = make_float2(pa.x, pa.y);
                p3[1] = make_float2(pa.z, pa.w);
                p3[2] = make_float2(pb.x, pb.y);
                q3[0] = make_float2(qa.x, qa.y);
                q3[1] = make_float2(qa.z, qa.w);
                q3[2] = make_float2(qb.x, qb.y);
                z3[0] = za.x;
                z3[1] = za.y;
                z3[2] = zb.x;
                b3[0] = ba.x;
                b3[1] = ba.y;
                b3[2] = bb.x;
            } else {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    p3[k] = s_exby[ei + ch + k];
                    q3[k] = s_eybx[eh + ci + k];
                    z3[k] = s_ez[ei + ci + k];
                    b3[k] = s_bz[eh + ch + k];
                }
            }
            const float pex = fmaf(hx3[0], p3[0].x, fmaf(hx3[1], p3[1].x, hx3[2] * p3[2].x));
            const float pby = fmaf(hx3[0], p3[0].y, fmaf(hx3[1], p3[1].y, hx3[2] * p3[2].y));
            const float qey = fmaf(ix3[0], q3[0].x, fmaf(ix3[1], q3[1].x, ix3[2] * q3[2].x));
            const float qbx = fmaf(ix3[0], q3[0].y, fmaf(ix3[1], q3[1].y, ix3[2] * q3[2].y));
            const float zz = fmaf(ix3[0], z3[0], fmaf(ix3[1], z3[1], ix3[2] * z3[2]));
            const float bz = fmaf(hx3[0], b3[0], fmaf(hx3[1], b3[1], hx3[2] * b3[2]));
            Ex = fmaf(iy3[r], pex, Ex);
            By = fmaf(iy3[r], pby, By);
            Ey = fmaf(hy3[r], qey, Ey);
            Bx = fmaf(hy3[r], qbx, Bx);
            Ez = fmaf(iy3[r], zz, Ez);
            Bz = fmaf(hy3[r], bz, Bz);
        }
    } else {
        // ---- interpolation (bilinear at each component's staggered point)
        const bool xh = x >= 0.5f, yh = y >= 0.5f;
        const float wxh = xh ? x - 0.5f : x + 0.5f;   // weight for (i+1/2) points
        const float wyh = yh ? y - 0.5f : y + 0.5f;
        const int ch = lx + (H - 1) + (xh ? 1 : 0);   // packed column of the half stencil
        const int rh = ly + (H - 1) + (yh ? 1 : 0);
        const int c0 = lx + H, r0 = ly + H;
        const int e0 = __mul24(r0, NE), eh = __mul24(rh, NE);
        // each stencil: the two x-neighbours on two rows (the values at cells
        // (c, c+1) of a row: one entry in the packed layout, two adjacent ones
        // -- one ds_read2 -- otherwise)
        if constexpr (std::is_same<V2, float4>::value) {
            const float4 p0 = s_exby[e0 + ch], p1 = s_exby[e0 + NE + ch];
            const float4 q0 = s_eybx[eh + c0], q1 = s_eybx[eh + NE + c0];
            const float2 z0 = s_ez[e0 + c0], z1 = s_ez[e0 + NE + c0];
            const float2 b0 = s_bz[eh + ch], b1 = s_bz[eh + NE + ch];
            Ex = lerpf(lerpf(p0.x, p0.z, wxh), lerpf(p1.x, p1.z, wxh), y);
            By = lerpf(lerpf(p0.y, p0.w, wxh), lerpf(p1.y, p1.w, wxh), y);
            Ey = lerpf(lerpf(q0.x, q0.z, x), lerpf(q1.x, q1.z, x), wyh);
            Bx = lerpf(lerpf(q0.y, q0.w, x), lerpf(q1.y, q1.w, x), wyh);
            Ez = lerpf(lerpf(z0.x, z0.y, x), lerpf(z1.x, z1.y, x), y);
            Bz = lerpf(lerpf(b0.x, b0.y, wxh), lerpf(b1.x, b1.y, wxh), wyh);
        } else {
            const float2 p0 = s_exby[e0 + ch], p0r = s_exby[e0 + ch + 1];
            const float2 p1 = s_exby[e0 + NE + ch], p1r = s_exby[e0 + NE + ch + 1];
            const float2 q0 = s_eybx[eh + c0], q0r = s_eybx[eh + c0 + 1];
            const float2 q1 = s_eybx[eh + NE + c0], q1r = s_eybx[eh + NE + c0 + 1];
            const float z0 = s_ez[e0 + c0], z0r = s_ez[e0 + c0 + 1], z1 = s_ez[e0 + NE + c0], z1r = s_ez[e0 + NE + c0 + 1];
            const float b0 = s_bz[eh + ch], b0r = s_bz[eh + ch + 1], b1 = s_bz[eh + NE + ch], b1r = s_bz[eh + NE + ch + 1];
            Ex = lerpf(lerpf(p0.x, p0r.x, wxh), lerpf(p1.x, p1r.x, wxh), y);
            By = lerpf(lerpf(p0.y, p0r.y, wxh), lerpf(p1.y, p1r.y, wxh), y);
            Ey = lerpf(lerpf(q0.x, q0r.x, x), lerpf(q1.x, q1r.x, x), wyh);
            Bx = lerpf(lerpf(q0.y, q0r.y, x), lerpf(q1.y, q1r.y, x), wyh);
            Ez = lerpf(lerpf(z0, z0r, x), lerpf(z1, z1r, x), y);
            Bz = lerpf(lerpf(b0, b0r, wxh), lerpf(b1, b1r, wxh), wyh);
        }
    }

    // ---- Boris push (Eqs. 6-10); 1 + |u|^2 >= 1, so the hardware
    // reciprocal square root needs no denormal care
    const float ux0 = p.ux, uy0 = p.uy, uz0 = p.uz;
    const float mx = fmaf(h, Ex, ux0), my = fmaf(h, Ey, uy0), mz = fmaf(h, Ez, uz0);
    const float gi = __builtin_amdgcn_rsqf(fmaf(mx, mx, fmaf(my, my, fmaf(mz, mz, 1.0f))));
    const float hg = h * gi;
    const float tx_ = hg * Bx, ty_ = hg * By, tz_ = hg * Bz;
    const float px = fmaf(my, tz_, fmaf(-mz, ty_, mx));
    const float py = fmaf(mz, tx_, fmaf(-mx, tz_, my));
    const float pz = fmaf(mx, ty_, fmaf(-my, tx_, mz));
    const float f2 = 2.0f * __builtin_amdgcn_rcpf(fmaf(tx_, tx_, fmaf(ty_, ty_, fmaf(tz_, tz_, 1.0f))));
    const float sx_ = f2 * tx_, sy_ = f2 * ty_, sz_ = f2 * tz_;
    const float ux = fmaf(h, Ex, fmaf(py, sz_, fmaf(-pz, sy_, mx)));
    const float uy = fmaf(h, Ey, fmaf(pz, sx_, fmaf(-px, sz_, my)));
    const float uz = fmaf(h, Ez, fmaf(px, sy_, fmaf(-py, sx_, mz)));

    // ---- move (Eq. 11), in cells
    const float ig = __builtin_amdgcn_rsqf(fmaf(ux, ux, fmaf(uy, uy, fmaf(uz, uz, 1.0f))));
    float dX = ux * ig * a.cx, dY = uy * ig * a.cy;
    const bool ok = fabsf(dX) < 1.0f && fabsf(dY) < 1.0f;
    if (valid && !ok) m.err |= kErrRange;
    dX = ok ? dX : 0.0f;
    dY = ok ? dY : 0.0f;
    const float x1 = x + dX, y1 = y + dY;
    const int sxn = x1 >= 1.0f ? 1 : (x1 < 0.0f ? -1 : 0);
    const int syn = y1 >= 1.0f ? 1 : (y1 < 0.0f ? -1 : 0);

    // ---- current: a motion inside its cell is one piece, and there both
    // deposits agree (x, x1 in [0, 1)); one that crosses a face is queued
    // whole and cut (or, for Esirkepov, spread over its 4 x 4 stencil) when
    // the queue is drained
    m.fqvz = fq * uz * ig;
    m.b = jcell<NJ, H>(lx, ly);
    if constexpr (DM == kDepQuad) {
        // quadratic shape: queued when the nearest node changes on an axis
        // (the shape then spans four nodes there)
        const bool nx = (x1 + 0.5f >= 1.0f) != (x >= 0.5f) || x1 + 0.5f < 0.0f || x1 + 0.5f >= 2.0f;
        const bool ny = (y1 + 0.5f >= 1.0f) != (y >= 0.5f) || y1 + 0.5f < 0.0f || y1 + 0.5f >= 2.0f;
        m.cross = valid && (nx || ny);
    } else {
        m.cross = valid && (sxn | syn) != 0;
    }
    m.x = x;
    m.y = y;
    m.dX = dX;
    m.dY = dY;

    // ---- new position: offset back into [0,1), cell index, periodic wrap.
    // A backward step whose offset rounds up to 1 lies on the face: it is
    // x = 0 of the old cell (likewise y).
    const float xs = sxn > 0 ? x1 - 1.0f : (sxn < 0 ? x1 + 1.0f : x1);
    const float ys = syn > 0 ? y1 - 1.0f : (syn < 0 ? y1 + 1.0f : y1);
    const bool xr = sxn < 0 && xs >= 1.0f, yr = syn < 0 && ys >= 1.0f;
    m.xn = xr ? 0.0f : xs;
    m.yn = yr ? 0.0f : ys;
    const int nlx = lx + sxn + (xr ? 1 : 0), nly = ly + syn + (yr ? 1 : 0);
    const int gx = wrapi(gx0 + nlx, a.nx), gy = wrapi(gy0 + nly, a.ny);
    m.ncell = gx | (gy << 16);
    // on an axis of one tile the periodic image is in the tile itself
    m.nlc = tcell_pack(tx_wrap ? nlx : gx, ty_wrap ? nly : gy);
    m.ux = ux;
    m.uy = uy;
    m.uz = uz;
    // the step to the new tile; on an axis of two tiles both neighbours are
    // the same tile, and the step is counted +1 either way
    const int dtx = tx_wrap ? (nlx < 0 ? (a.ntx == 2 ? 1 : -1) : (nlx >= T ? 1 : 0)) : 0;
    const int dty = ty_wrap ? (nly < 0 ? (a.nty == 2 ? 1 : -1) : (nly >= T ? 1 : 0)) : 0;
    m.dir = (dty + 1) * 3 + (dtx + 1);
    return m;
}

// One tile of one simulation, by the whole workgroup (push_waves(T) wavefronts).
// C: particles per lane per pass of the particle loop (64-particle chunks
// carried side by side).
template <int T, int R, int JM, int DM, int H, int C, bool MS = false>
__device__ __forceinline__ void push_tile(const PushArgs &a, const int tile, const bool rebase)
{
    static_assert(cadence_ok(T, H), "halo pad not supported for this tile");
    constexpr int NE = T + 2 * H;       // staged E/B cells per axis: relative -H..T+H-1
    constexpr int NJ = T + 2 * H + 1;   // current halo nodes per axis: relative -H..T+H
    constexpr int JP = NJ * NJ;
    constexpr int W = push_waves(T);   // wavefronts of the workgroup
    constexpr int NT = 64 * W;         // its threads
    using Acc = typename JAcc<JM>::T;

    // E/B halo: entry [r][c] holds relative cell (c-H, r-H) -- and, in the
    // packed layout, cell (c-H+1, r-H) after it; the two components
    // interpolated at the same points share an entry
    constexpr bool P = push_packed(T);
    using V2 = typename std::conditional<P, float4, float2>::type;
    using V1 = typename std::conditional<P, float2, float>::type;
    __shared__ V2 s_exby[NE * NE];   // Ex, By (packed: Ex, By, Ex', By')
    __shared__ V2 s_eybx[NE * NE];   // Ey, Bx
    __shared__ V1 s_ez[NE * NE];
    __shared__ V1 s_bz[NE * NE];
    __shared__ uint32_t s_lb[P ? W : 1][7][P ? kLeaverBuf : 1];   // packed layout: leaver entry + new data
    __shared__ Acc s_j[R][3 * JP];
    __shared__ int s_dir[kMaxSpecies][9];
    __shared__ int s_wl[kMaxSpecies][W];
    __shared__ uint32_t s_pq[W][6][kMotionBuf];   // queued face-crossing motions
    __shared__ int s_fill[W][64];                  // pending holes of the chunk being loaded

    const int tx = tile % a.ntx, ty = tile / a.ntx;
    const int gx0 = tx * T, gy0 = ty * T;
    const int tid = threadIdx.x;
    // the wavefront index is uniform across the wavefront: keep it (and the
    // buffer descriptors derived from it) in scalar registers
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t plane = (int64_t)a.nx * a.ny;

    for (int e = tid; e < NE * NE; e += NT) {
        const int r = e / NE, c = e - r * NE;
        const int64_t row = (int64_t)wrapi(gy0 - H + r, a.ny) * a.nx;
        const int64_t i0 = row + wrapi(gx0 - H + c, a.nx);
        const PIC_GLOBAL float *f = gp(a.fld);
        if constexpr (P) {
            const int64_t i1 = row + wrapi(gx0 - H + 1 + c, a.nx);
            s_exby[e] = make_float4(f[i0], f[4 * plane + i0], f[i1], f[4 * plane + i1]);
            s_eybx[e] = make_float4(f[plane + i0], f[3 * plane + i0], f[plane + i1], f[3 * plane + i1]);
            s_ez[e] = make_float2(f[2 * plane + i0], f[2 * plane + i1]);
            s_bz[e] = make_float2(f[5 * plane + i0], f[5 * plane + i1]);
        } else {
            s_exby[e] = make_float2(f[i0], f[4 * plane + i0]);
            s_eybx[e] = make_float2(f[plane + i0], f[3 * plane + i0]);
            s_ez[e] = f[2 * plane + i0];
            s_bz[e] = f[5 * plane + i0];
        }
    }
    for (int e = tid; e < R * 3 * JP; e += NT) (&s_j[0][0])[e] = Acc(0);
    if (tid < kMaxSpecies * 9) (&s_dir[0][0])[tid] = 0;
    __syncthreads();

    Acc *sj = s_j[R > 1 ? lane % R : 0];
    const bool tx_wrap = a.ntx > 1, ty_wrap = a.nty > 1;
    // MS: the simulation's sort is the motion-class one, whose last pass --
    // the staging arrays copied back -- may have been left to this push: the
    // particles are then read from the staging arrays (the flag is cleared
    // by the next launch after this kernel)
    bool from_stg = false;
    if constexpr (MS) from_stg = *gp(a.stg_live) != 0;

    for (int s = 0; s < a.n_species; ++s) {
        const SpeciesDev sp = a.sp[s];
        const int begin = gp(sp.off)[tile], end = gp(sp.off)[tile + 1];
        int lo, hi;
        wave_range(begin, end, wave, W, lo, hi);
        int nleav = 0;   // wavefront-uniform
        if (lo < hi) {
            // buffer views from the first 64-aligned slot of the section to the
            // end of this wavefront's run: loads beyond it (the prefetch past
            // the last chunk, the tail lanes of that chunk) return 0 without
            // touching memory
            const int base = (begin >> 6) << 6;
            const int bytes = (hi - base) * 4;
            const Stream6 st = stream6(sp.cell, sp.x, sp.y, sp.ux, sp.uy, sp.uz, base, bytes);   // the particle arrays
            // MS: the loads' view, the staging arrays or the same
            const Stream6 ld = MS && from_stg ? stream6(sp.scell, sp.sx, sp.sy, sp.sux, sp.suy, sp.suz, base, bytes)
                                              : st;
            const float h = sp.h, fq = sp.fq;
            // The fill the last sort left (holes of the section, ascending,
            // whose particles wait in the staging records): a window of 64 of
            // this run's hole slots, one per lane (fhw: the slot of rank
            // fhb + lane), the next rank not yet placed (fhp) and its slot
            // (fnext, INT_MAX once none is left).  All uniform but fhw.
            const int nfill = gp(sp.fcount)[tile];
            const PIC_GLOBAL int32_t *fhole = gp(sp.fhole) + begin;
            int fhb = 0, fhp = 0, fhw = INT_MAX, fnext = INT_MAX;
            if (nfill > 0) {
                fhb = fhp = gp(sp.fbase)[(int64_t)tile * W + wave];
                fhw = fhb + lane < nfill ? fhole[fhb + lane] : INT_MAX;
                fnext = fhp < nfill ? __builtin_amdgcn_readfirstlane(fhw) : INT_MAX;
            }
            // the rank of the hole at slot c0 + lane (chunks in ascending
            // order), or -1; `any` (uniform): the chunk has a hole.  A chunk
            // without holes costs one compare
            auto fill_ref = [&](int c0, bool &any) -> int {
                const int lim = min(c0 + 64, hi);
                any = fnext < lim;
                if (!any) return -1;
                int *map = s_fill[wave];
                map[lane] = -1;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                for (;;) {
                    const bool in = lane >= fhp - fhb && fhw >= c0 && fhw < lim;
                    const unsigned long long mk = __ballot(in);
                    if (in) map[fhw - c0] = fhb + lane;
                    fhp += __popcll(mk);
                    if (fhp - fhb < 64 || fhp >= nfill) break;
                    fhb = fhp;   // the window is used up: the next one
                    fhw = fhb + lane < nfill ? fhole[fhb + lane] : INT_MAX;
                    if (__builtin_amdgcn_readfirstlane(fhw) >= lim) break;
                }
                fnext = fhp < nfill ? __builtin_amdgcn_readlane(fhw, fhp - fhb) : INT_MAX;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                return map[lane];
            };
            // a hole lane's particle from its staged 32-byte record
            auto fill_load = [&](Chunk &d, int ref) {
                if (ref >= 0) {
                    const PIC_GLOBAL vf4 *r = (const PIC_GLOBAL vf4 *)(sp.fsrc + begin + ref);
                    const vf4 u = r[0];
                    const vf2 v = *(const PIC_GLOBAL vf2 *)(r + 1);
                    const int g = __float_as_int(u.x);   // a particle of this tile, whole-grid cell
                    d.cell = tcell_pack((g & 0xffff) - gx0, (g >> 16) - gy0);
                    d.x = u.y;
                    d.y = u.z;
                    d.ux = u.w;
                    d.uy = v.x;
                    d.uz = v.y;
                }
            };
            int npq = 0;    // motions waiting in the wavefront's queue (uniform)
            int nbuf = 0;   // leavers waiting in the wavefront's LDS buffer (packed layout; uniform)
            // C chunks per iteration: lane L holds the particles of slots
            // cb + L, cb + 64 + L, ...  Their arithmetic (advance) has no side
            // effects and no branches, so the C instruction streams
            // interleave; the side effects (finish) follow in slot order.
            // Loads past the run's end return 0; lanes before its start (first
            // chunk of the section only) read the previous tile's particles
            // and discard them.  The next C chunks are always prefetched
            // before the current ones are processed.
            auto finish = [&](const Moved &m, int i, int at) {
                if constexpr (DM == kDepQuad) {
                    if (m.valid && !m.cross)
                        deposit_quad3<NJ, JM>(sj, m.b, m.x >= 0.5f ? 1 : 0, m.y >= 0.5f ? 1 : 0, m.x, m.y, m.dX,
                                              m.dY, m.fqvz, fq);
                } else {
                    if (m.valid && !m.cross) deposit_piece<NJ, JM>(sj, m.b, m.x, m.y, m.dX, m.dY, m.fqvz, fq);
                }
                if (m.valid) {
                    __builtin_amdgcn_raw_buffer_store_b16((unsigned short)m.nlc, st.cell, at >> 1, 0, kStoreCpol);
                    stf(st.x, at, m.xn);
                    stf(st.y, at, m.yn);
                    stf(st.ux, at, m.ux);
                    stf(st.uy, at, m.uy);
                    stf(st.uz, at, m.uz);
                }
                queue_motion<NJ, JM, DM>(sj, s_pq[wave], npq, m.cross, m.b, m.x, m.y, m.dX, m.dY, m.fqvz, fq,
                                         lane);
                // leavers are appended to the wavefront's leaver sub-list in
                // slot order, with a copy of their new data: through the
                // wavefront's LDS buffer, written out as whole lines (packed
                // layout), or straight from the registers
                const bool leaver = m.valid && m.dir != 4;
                const unsigned long long mk = __ballot(leaver);
                if constexpr (P) {
                    const int c = __popcll(mk);
                    if (c != 0) {
                        if (nbuf + c > kLeaverBuf) {
                            flush_leavers(sp, s_lb[wave], nbuf, (int64_t)lo + nleav, lane);
                            nleav += nbuf;
                            nbuf = 0;
                        }
                        if (leaver) {
                            const int r = nbuf + lane_rank(mk);
                            s_lb[wave][0][r] = ((uint32_t)(i - begin) << 4) | (uint32_t)m.dir;
                            s_lb[wave][1][r] = (uint32_t)m.ncell;
                            s_lb[wave][2][r] = __float_as_uint(m.xn);
                            s_lb[wave][3][r] = __float_as_uint(m.yn);
                            s_lb[wave][4][r] = __float_as_uint(m.ux);
                            s_lb[wave][5][r] = __float_as_uint(m.uy);
                            s_lb[wave][6][r] = __float_as_uint(m.uz);
                            atomicAdd(&s_dir[s][m.dir], 1);
                        }
                        nbuf += c;
                    }
                } else {
                    if (leaver) {
                        const int64_t q = (int64_t)lo + nleav + lane_rank(mk);
                        gp(sp.leav)[q] = ((uint32_t)(i - begin) << 4) | (uint32_t)m.dir;
                        put_leaver(sp.lrec, q, m.ncell, m.xn, m.yn, m.ux, m.uy, m.uz);
                        atomicAdd(&s_dir[s][m.dir], 1);
                    }
                    nleav += __popcll(mk);
                }
            };
            int cb = (lo >> 6) << 6;
            int off = (cb + lane - base) * 4;
            Chunk nxt[C], nstg[C];
            int nref[C];
            bool nany[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                nxt[c] = load_chunk(ld, off + 256 * c);
                nref[c] = fill_ref(cb + 64 * c, nany[c]);
                nstg[c] = Chunk{};
                fill_load(nstg[c], nref[c]);
            }
            int errs = 0;   // error bits of this lane's particles
            for (; cb < hi; cb += 64 * C, off += 256 * C) {
                Chunk cur[C];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    cur[c] = nxt[c];
                    if (nany[c] && nref[c] >= 0) cur[c] = nstg[c];   // a hole: its particle from the fill
                    nxt[c] = load_chunk(ld, off + 256 * (C + c));
                    nref[c] = fill_ref(cb + 64 * (C + c), nany[c]);
                    fill_load(nstg[c], nref[c]);
                }
                const int i = cb + lane;
                Moved m[C];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    m[c] = advance<T, NJ, NE, H, DM, V2, V1>(a, cur[c], i + 64 * c >= lo && i + 64 * c < hi, rebase,
                                                         gx0, gy0, tx_wrap, ty_wrap, h, fq, s_exby, s_eybx, s_ez,
                                                         s_bz);
                    errs |= m[c].err;
                }
#pragma unroll
                for (int c = 0; c < C; ++c) finish(m[c], i + 64 * c, off + 256 * c);
            }
            if (errs) set_err(a.err, errs);
            drain_motions<NJ, JM, DM>(sj, s_pq[wave], npq, fq, lane);
            if constexpr (P) {
                flush_leavers(sp, s_lb[wave], nbuf, (int64_t)lo + nleav, lane);
                nleav += nbuf;
            }
        }
        if (lane == 0) s_wl[s][wave] = nleav;
    }
    __syncthreads();
    // the fill the last sort left is done (every wavefront has read its count)
    if (tid < a.n_species && gp(a.sp[tid].fcount)[tile] != 0) gp(a.sp[tid].fcount)[tile] = 0;

    // the int64 current sums are exact while the tile holds fewer than 2^31
    // particles over all species
    if (JM == kJFixed && tid == 0) {
        int64_t total = 0;
        for (int s = 0; s < a.n_species; ++s) total += gp(a.sp[s].off)[tile + 1] - gp(a.sp[s].off)[tile];
        if (total >= (int64_t(1) << 31)) set_err(a.err, kErrOverflow);
    }
    // per-tile count records
    if (tid < a.n_species * kCntStride) {
        const int s = tid / kCntStride, k = tid % kCntStride;
        const int n = gp(a.sp[s].off)[tile + 1] - gp(a.sp[s].off)[tile];
        int leavers = 0;
        for (int w = 0; w < W; ++w) leavers += s_wl[s][w];
        int v = 0;
        if (k < 9) v = (k == 4) ? n - leavers : s_dir[s][k];
        else if (k == kCntLeavers) v = leavers;
        else if (k < kCntSub + W) v = s_wl[s][k - kCntSub];
        gp(a.sp[s].cnt)[(int64_t)tile * kCntStride + k] = v;
    }

    // the tile's current halo in physical units
    PIC_GLOBAL float *out = gp(a.jtile) + (int64_t)tile * 3 * JP;
    for (int e = tid; e < 3 * JP; e += NT) {
        const int comp = e / JP;
        out[e] = JAcc<JM>::value(&s_j[0][e], R, 3 * JP, a.ju[comp], a.err);
    }
    // The first half step of the field advance for the tile's own cells, from
    // the staged halo (cell (i, j) is entry (j + H) NE + i + H; its +x and +y
    // neighbours are in the halo since H >= 1), into the half-step planes.
    if (a.bh) {
        PIC_GLOBAL float *bh = gp(a.bh);
        for (int c = tid; c < T * T; c += NT) {
            const int i = c % T, j = c / T;
            const int e = (j + H) * NE + (i + H);
            float ex, ex_y, ey, ey_x, ez, ez_x, ez_y, bx, by, bz;
            if constexpr (P) {   // entries hold cells i and i + 1
                const float4 q = s_exby[e], w = s_eybx[e];
                const float2 z = s_ez[e];
                ex = q.x;
                by = q.y;
                ex_y = s_exby[e + NE].x;
                ey = w.x;
                bx = w.y;
                ey_x = w.z;
                ez = z.x;
                ez_x = z.y;
                ez_y = s_ez[e + NE].x;
                bz = s_bz[e].x;
            } else {
                const float2 q = s_exby[e], w = s_eybx[e];
                ex = q.x;
                by = q.y;
                ex_y = s_exby[e + NE].x;
                ey = w.x;
                bx = w.y;
                ey_x = s_eybx[e + 1].x;
                ez = s_ez[e];
                ez_x = s_ez[e + 1];
                ez_y = s_ez[e + NE];
                bz = s_bz[e];
            }
            const BCell b = faraday_half(bx, by, bz, ex, ex_y, ey, ey_x, ez, ez_x, ez_y, a.hdx, a.hdy);
            const int64_t g = (int64_t)(gy0 + j) * a.nx + (gx0 + i);
            bh[g] = b.x;
            bh[plane + g] = b.y;
            bh[2 * plane + g] = b.z;
        }
    }

}

// Register budget: the LDS fit (push_min_waves), and at most two waves per
// SIMD (256 VGPRs) for four chunks per lane, whose particle state does not
// fit 128 registers.
template <int T, int R, int JM, int DM, int H, int C>
constexpr int push_waves_per_simd()
{
    return C > 2 && push_min_waves(T, R, JM, H) > 2 ? 2 : push_min_waves(T, R, JM, H);
}

template <int T, int R, int JM, int DM, int H, int C, bool MS>
__global__ void __launch_bounds__(64 * push_waves(T), (push_waves_per_simd<T, R, JM, DM, H, C>())) k_push_deposit(PushArgs a)
{
    push_tile<T, R, JM, DM, H, C, MS>(a, blockIdx.x, a.rebase != 0);
}

// Many simulations in one launch: one workgroup per (simulation, tile) item.
// The items come largest simulations first and the hardware dispatches
// workgroups in order, so the expensive tiles start early and the cheap ones
// fill the tail.  (A persistent grid taking items from a shared counter keeps
// the counter, the item table and the descriptor pointer live across the
// whole tile loop: more scalar registers than the push has, spilled.)
template <int T, int R, int JM, int DM, int H, int C>
__global__ void __launch_bounds__(64 * push_waves(T), (push_waves_per_simd<T, R, JM, DM, H, C>())) k_push_batch(const PushArgs *__restrict__ descs,
                                                       const int4 *__restrict__ items, int n_items, int rebase)
{
    if ((int)blockIdx.x >= n_items) return;
    const int4 w = items[blockIdx.x];
    push_tile<T, R, JM, DM, H, C>(descs[w.x], w.y, rebase != 0);
}

// The periodic fold of the tile current halos into the J planes
// (update_gc_add), one 64 x 4 block of nodes; the per-node sum is fold_node
// (pic_fold.h), which the fused field advance shares.
template <int T, int H>
__device__ __forceinline__ void j_reduce_block(const JReduceArgs &r, int bxb, int byb)
{
    const int nx = r.nx, ny = r.ny;
    const int gx = bxb * 64 + (threadIdx.x & 63);
    const int gy = byb * 4 + (threadIdx.x >> 6);
    if (gx >= nx || gy >= ny) return;
    float j[3];
    fold_node<T, H>(r.jtile, nx, ny, r.ntx, r.nty, gx, gy, j);
    const int64_t plane = (int64_t)nx * ny;
    const int64_t k = (int64_t)gy * nx + gx;
    float *__restrict__ J = r.J;
    J[k] = j[0];
    J[plane + k] = j[1];
    J[2 * plane + k] = j[2];
}

template <int T, int H>
__global__ void __launch_bounds__(256) k_j_reduce(JReduceArgs r)
{
    j_reduce_block<T, H>(r, blockIdx.x, blockIdx.y);
}

// node blocks of many simulations: items = (simulation, bx, by)
template <int T, int H>
__global__ void __launch_bounds__(256) k_j_reduce_batch(const JReduceArgs *__restrict__ descs,
                                                        const int4 *__restrict__ items)
{
    const int4 w = items[blockIdx.x];
    j_reduce_block<T, H>(descs[w.x], w.y, w.z);
}

template <int T, int R, int JM, int DM, int H, int C, bool MS>
static void launch_pd(const PushArgs &a, int n_tiles, hipStream_t s)
{
    hipLaunchKernelGGL((k_push_deposit<T, R, JM, DM, H, C, MS>), dim3(n_tiles), dim3(64 * push_waves(T)), 0, s, a);
}

template <int T, int R, int JM, int DM, int H, int C>
static void launch_pb(const PushArgs *descs, const int4 *items, int n_items, int rebase, hipStream_t s)
{
    hipLaunchKernelGGL((k_push_batch<T, R, JM, DM, H, C>), dim3(n_items), dim3(64 * push_waves(T)), 0, s, descs,
                       items, n_items, rebase);
}

// One push launch, single or batched, with every template parameter chosen.
// Configurations over the LDS budget or outside cadence_ok are rejected by
// pic_query / pic_init / pic_batch_init; they launch nothing here.
struct PushLaunch {
    const PushArgs *single;   // single simulation (n_tiles workgroups), or null
    int n_tiles;
    const PushArgs *descs;    // batched: one workgroup per item
    const int4 *items;
    int n_items;
    int rebase;               // batched: the pushes follow a sort
    int ms;                   // single: the particles may wait in the motion-class sort's staging arrays
    hipStream_t s;
    template <int T, int R, int JM, int DM, int H, int C>
    void go() const
    {
        if constexpr (push_lds_bytes(T, R, JM, H) <= kLdsBytes && cadence_ok(T, H)) {
            if (single) {
                // the reading of the staging arrays is built for the default current and deposit
                if constexpr (R == 1 && JM == kJFixed && DM == kDepVB) {
                    if (ms) {
                        launch_pd<T, R, JM, DM, H, C, true>(*single, n_tiles, s);
                        return;
                    }
                }
                launch_pd<T, R, JM, DM, H, C, false>(*single, n_tiles, s);
            } else {
                launch_pb<T, R, JM, DM, H, C>(descs, items, n_items, rebase, s);
            }
        }
    }
};

// particles per lane per pass: 1, 2 or 4 for the default current and
// deposit with one LDS copy (the configurations the autotuner searches), 1
// for the quadratic shape, 2 otherwise (pic_query / pic_init refuse the rest)
template <int T, int R, int JM, int DM, int H>
static void push_c(const PushLaunch &L, int ppl)
{
    if constexpr (DM == kDepQuad) {
        // one chunk per lane: the nine-point stencils of two particles in
        // flight would not fit the register budget
        L.go<T, R, JM, DM, H, 1>();
        return;
    }
    if constexpr (R == 1 && JM == kJFixed && DM == kDepVB) {
        if (ppl == 1) {
            L.go<T, R, JM, DM, H, 1>();
            return;
        }
        if (ppl == 4) {
            L.go<T, R, JM, DM, H, 4>();
            return;
        }
    }
    L.go<T, R, JM, DM, H, 2>();
}

template <int T, int JM, int DM>
static void push_r(const PushLaunch &L, int replicas, int halo, int ppl)
{
    if constexpr (DM == kDepQuad) {
        // the quadratic shape: one sort per step, halo pad 2, one LDS copy
        if (halo == 2) push_c<T, 1, JM, DM, 2>(L, ppl);
        return;
    }
    if (halo > 1) {
        // sort cadences above 1: fixed-point current, one LDS copy
        if constexpr (JM == kJFixed) {
            if (halo == 2) push_c<T, 1, JM, DM, 2>(L, ppl);
            else push_c<T, 1, JM, DM, 4>(L, ppl);
        }
        return;
    }
    switch (replicas) {
    case 1: push_c<T, 1, JM, DM, 1>(L, ppl); break;
    case 2: push_c<T, 2, JM, DM, 1>(L, ppl); break;
    default: push_c<T, 4, JM, DM, 1>(L, ppl); break;
    }
}

// the Esirkepov deposit (linear or quadratic shape) is built for the
// fixed-point current only
template <int T>
static void push_j(const PushLaunch &L, int replicas, int jmode, int dmode, int halo, int ppl)
{
    if (jmode == kJFloat) push_r<T, kJFloat, kDepVB>(L, replicas, halo, ppl);
    else if (dmode == kDepQuad) push_r<T, kJFixed, kDepQuad>(L, replicas, halo, ppl);
    else if (dmode == kDepEsirkepov) push_r<T, kJFixed, kDepEsirkepov>(L, replicas, halo, ppl);
    else push_r<T, kJFixed, kDepVB>(L, replicas, halo, ppl);
}

static void push_t(const PushLaunch &L, int tile, int replicas, int jmode, int dmode, int halo, int ppl)
{
    switch (tile) {
    case 8: push_j<8>(L, replicas, jmode, dmode, halo, ppl); break;
    case 16: push_j<16>(L, replicas, jmode, dmode, halo, ppl); break;
    default: push_j<32>(L, replicas, jmode, dmode, halo, ppl); break;
    }
}

void launch_push_deposit(int tile, int replicas, int jmode, int dmode, int halo, int ppl, const PushArgs &a,
                         int n_tiles, bool ms, hipStream_t s)
{
    PushLaunch L{&a, n_tiles, nullptr, nullptr, 0, 0, ms ? 1 : 0, s};
    push_t(L, tile, replicas, jmode, dmode, halo, ppl);
}

void launch_push_batch(int tile, int replicas, int jmode, int dmode, int halo, int ppl, const PushArgs *descs,
                       const int4 *items, int n_items, bool rebase, hipStream_t s)
{
    PushLaunch L{nullptr, 0, descs, items, n_items, rebase ? 1 : 0, 0, s};
    push_t(L, tile, replicas, jmode, dmode, halo, ppl);
}

template <int T>
static void jr_h(int halo, const JReduceArgs *single, const JReduceArgs *descs, const int4 *items, int n_items,
                 hipStream_t s)
{
    auto go = [&](auto hc) {
        constexpr int H = decltype(hc)::value;
        if constexpr (cadence_ok(T, H)) {
            if (single) {
                dim3 grid((single->nx + 63) / 64, (single->ny + 3) / 4);
                hipLaunchKernelGGL((k_j_reduce<T, H>), grid, dim3(256), 0, s, *single);
            } else {
                hipLaunchKernelGGL((k_j_reduce_batch<T, H>), dim3(n_items), dim3(256), 0, s, descs, items);
            }
        }
    };
    if (halo == 2) go(std::integral_constant<int, 2>());
    else if (halo == 4) go(std::integral_constant<int, 4>());
    else go(std::integral_constant<int, 1>());
}

static void jr_t(int tile, int halo, const JReduceArgs *single, const JReduceArgs *descs, const int4 *items,
                 int n_items, hipStream_t s)
{
    switch (tile) {
    case 8: jr_h<8>(halo, single, descs, items, n_items, s); break;
    case 16: jr_h<16>(halo, single, descs, items, n_items, s); break;
    default: jr_h<32>(halo, single, descs, items, n_items, s); break;
    }
}

void launch_j_reduce(int tile, int halo, const JReduceArgs &r, hipStream_t s)
{
    jr_t(tile, halo, &r, nullptr, nullptr, 0, s);
}

void launch_j_reduce_batch(int tile, int halo, const JReduceArgs *descs, const int4 *items, int n_items,
                           hipStream_t s)
{
    if (n_items == 0) return;
    jr_t(tile, halo, nullptr, descs, items, n_items, s);
}

__global__ void k_set_int(int *p, int v) { *p = v; }

void launch_set_int(int *p, int v, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, p, v);
}

}  // namespace pic

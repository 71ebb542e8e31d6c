// Strict re-sort of particles by tile (Sec. 4.3, the bucket sort of Fig. 4.5),
// redesigned for gfx950: no atomics decide any position, so the permutation
// is the canonical one and is reproducible bit for bit.
//
//   k_sort_count, k_sort_add_direct (k_sort_scan_blocks, k_sort_add_base
//                  above 64 scan blocks)
//                  step (1): the new count of tile t is the sum, over the nine
//                  tiles a particle can come from, of the direction counts the
//                  push kernel recorded; an exclusive scan gives tile_offset'.
//   k_sort_plan    steps (2)-(4), one wavefront per destination tile t with
//                  new section [A, B):
//                    holes  = slots of [A, B) whose particle is not in tile t,
//                             in ascending order: the parts of [A, B) outside
//                             t's old section (read the cells there) and t's
//                             own leavers inside it (from its leaver lists);
//                    movers = particles of tile t outside [A, B), ascending:
//                             the leavers of the up-to-eight neighbour tiles
//                             heading to t (their leaver lists) and t's own
//                             stayers pushed out of [A, B) by section shifts;
//                  every mover is copied, in hole order, to a staging area
//                  (contiguous stores), so only O(movers) particle bytes
//                  are touched and no particle slot is written while other
//                  plans may still read it.
//   k_sort_scatter step (5): the staged movers into their holes -- or, in
//                  pic_step, nothing: the next push fills each hole from
//                  the staging area as it streams its section (a deferred
//                  fill; k_fill completes one on its own when anything else
//                  is to read the particles first).
//
// The cells the kernels keep are 16-bit offsets from the tile whose section
// holds the particle (tcell_pack); the staging records carry whole-grid
// cells, converted on the way in and out.  Also here: the motion-class sort
// (the alternative of Sec. 4.3), the conversions between the caller's
// whole-grid cells and the 16-bit ones, and the tile offsets of caller
// particles at initialisation.
#include "pic_internal.h"

namespace pic {


__device__ __forceinline__ int wrap_s(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ int lane_rank_s(unsigned long long m)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// Exclusive scan of one int per thread over a 1024-thread block; returns the
// thread's prefix and writes the block total to *total.
__device__ int block_exclusive_scan_1024(int v, int *total)
{
    __shared__ int s_w[16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    if (w == 0) {
        int t = lane < 16 ? s_w[lane] : 0;
#pragma unroll
        for (int d = 1; d < 16; d <<= 1) {
            const int y = __shfl_up(t, d, 64);
            if (lane >= d) t += y;
        }
        if (lane < 16) s_w[lane] = t;
    }
    __syncthreads();
    const int base = w > 0 ? s_w[w - 1] : 0;
    *total = s_w[15];
    return base + x - v;
}

__device__ __forceinline__ int tile_count_in(const int32_t *cnt, int t, int ntx, int nty)
{
    const int tx = t % ntx, ty = t / ntx;
    int v = 0;
#pragma unroll
    for (int o = 0; o < 9; ++o) {
        const int odx = o % 3 - 1, ody = o / 3 - 1;
        const int src = wrap_s(ty - ody, nty) * ntx + wrap_s(tx - odx, ntx);
        v += cnt[(int64_t)src * kCntStride + o];
    }
    return v;
}

// Step (1), first pass: new count of every tile and its exclusive prefix
// within its block of kScanBlock tiles, in place of tile_offset (which goes
// to offp, the plan's old sections); block totals to bsum.
__device__ __forceinline__ void sort_count_unit(const SortArgs &a, int spi, int blk)
{
    const SortSpecies &sp = a.sp[spi];
    const int n_tiles = a.n_tiles;
    const int t = blk * kScanBlock + threadIdx.x;
    int c = t < n_tiles ? tile_count_in(sp.cnt, t, a.ntx, a.nty) : 0;
    if (t < n_tiles && sp.inj_off) c += sp.inj_off[t + 1] - sp.inj_off[t];   // the window's new particles
    // block exclusive scan (kScanBlock = 256: four wavefronts)
    __shared__ int s_w[kScanBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    int base = 0;
    for (int k = 0; k < w; ++k) base += s_w[k];
    if (t < n_tiles) {
        sp.offp[t] = sp.off[t];
        sp.off[t] = base + x - c;
    }
    if (t == n_tiles - 1) sp.offp[n_tiles] = sp.off[n_tiles];
    if (threadIdx.x == kScanBlock - 1) sp.bsum[blk] = base + x;
}

// Step (1), second pass (one block per species): exclusive scan of the block
// totals in place; tile_offset'[n_tiles] = total, checked against n.
__device__ __forceinline__ void sort_scan_unit(const SortArgs &a, int spi)
{
    const SortSpecies &sp = a.sp[spi];
    const int n_tiles = a.n_tiles;
    const int nb = (n_tiles + kScanBlock - 1) / kScanBlock;
    int carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 1024) {
        const int b = b0 + threadIdx.x;
        const int v = b < nb ? sp.bsum[b] : 0;
        int total;
        const int ex = block_exclusive_scan_1024(v, &total);
        if (b < nb) sp.bsum[b] = carry + ex;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sp.off[n_tiles] = carry;
        const int expect = sp.removed ? sp.n - *sp.removed + sp.inj_n : sp.n;
        if (carry != expect) atomicOr(a.err, kErrCount);
    }
}

// Step (1), third pass: add each block's base.
__device__ __forceinline__ void sort_add_unit(const SortArgs &a, int spi, int blk)
{
    const SortSpecies &sp = a.sp[spi];
    const int t = blk * kScanBlock + threadIdx.x;
    if (t < a.n_tiles) sp.off[t] += sp.bsum[blk];
}

// Step (1), second and third pass in one, while there are at most
// kScanDirect blocks: each block sums its predecessors' totals itself and
// adds them; the last one also writes tile_offset'[n_tiles] and checks it.
constexpr int kScanDirect = 64;
static_assert(kScanDirect <= kScanBlock, "one predecessor total per thread");
__device__ __forceinline__ void sort_add_direct_unit(const SortArgs &a, int spi, int blk)
{
    const SortSpecies &sp = a.sp[spi];
    const int n_tiles = a.n_tiles;
    const int nb = (n_tiles + kScanBlock - 1) / kScanBlock;
    __shared__ int s_w[kScanBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int v = (int)threadIdx.x < blk ? sp.bsum[threadIdx.x] : 0;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if (lane == 0) s_w[w] = v;
    __syncthreads();
    int base = 0;
#pragma unroll
    for (int k = 0; k < kScanBlock / 64; ++k) base += s_w[k];
    const int t = blk * kScanBlock + threadIdx.x;
    if (t < n_tiles) sp.off[t] += base;
    if (blk == nb - 1 && threadIdx.x == 0) {
        const int total = base + sp.bsum[blk];
        sp.off[n_tiles] = total;
        const int expect = sp.removed ? sp.n - *sp.removed + sp.inj_n : sp.n;
        if (total != expect) atomicOr(a.err, kErrCount);
    }
}

// Slot of the list holding flat index k, over the lists described by lanes
// 0..63 (exclusive prefix `ex` of their lengths, INT_MAX past the last list):
// the largest L with ex_L <= k.  Fixed-step binary search, all lanes active.
__device__ __forceinline__ int find_list(int k, int ex)
{
    int lo = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
        const int e = __shfl(ex, lo + step < 64 ? lo + step : 63, 64);
        if (lo + step < 64 && e <= k) lo += step;
    }
    return lo;
}

// Wave-wide exclusive prefix of v (and the total).
__device__ __forceinline__ int wave_exclusive(int v, int &total)
{
    const int lane = threadIdx.x & 63;
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    total = __shfl(x, 63, 64);
    return x - v;
}

// One particle's six values in registers.
struct Chunk6 {
    int cell;
    float x, y, ux, uy, uz;
};

// one leaver record (two vector loads)
__device__ __forceinline__ Chunk6 load_leaver(const LeaverRec *src, int64_t i)
{
    const PIC_GLOBAL vf4 *s = (const PIC_GLOBAL vf4 *)(src + i);
    const vf4 a = s[0];
    const vf2 b = *(const PIC_GLOBAL vf2 *)(s + 1);
    return Chunk6{__float_as_int(a.x), a.y, a.z, a.w, b.x, b.y};
}

// The particle at slot i, inside the tile whose first cell is (gx0, gy0),
// with its whole-grid cell (the staging records' form); mask: T - 1 in a
// sorted state (the cell is relative to the tile modulo T), else -1.
__device__ __forceinline__ Chunk6 load_parts(const Parts &src, int64_t i, int gx0, int gy0, int mask)
{
    const int lc = src.cell[i];
    return Chunk6{(gx0 + (tcell_x(lc) & mask)) | ((gy0 + (tcell_y(lc) & mask)) << 16), src.x[i], src.y[i],
                  src.ux[i], src.uy[i], src.uz[i]};
}

// A particle of the tile whose first cell is (gx0, gy0), given with its
// whole-grid cell, into slot j (its cell relative to that tile).
__device__ __forceinline__ void store_parts(const Parts &dst, int64_t j, const Chunk6 &c, int gx0, int gy0)
{
    dst.cell[j] = (int16_t)tcell_pack((c.cell & 0xffff) - gx0, (c.cell >> 16) - gy0);
    dst.x[j] = c.x;
    dst.y[j] = c.y;
    dst.ux[j] = c.ux;
    dst.uy[j] = c.uy;
    dst.uz[j] = c.uz;
}

// Whether tile-relative cell lc lies inside its tile (of edge T).
__device__ __forceinline__ bool tcell_inside(int lc, int T)
{
    return (unsigned)tcell_x(lc) < (unsigned)T && (unsigned)tcell_y(lc) < (unsigned)T;
}

// Steps (2)-(4) of the sort for one destination tile t per wavefront, new
// section [A, B), old section [oA, oB).  Every candidate list of holes and
// of movers is described by one list slot (two per lane: slots lane and
// lane + 64); the lists are streamed as one flat index space, holes first,
// and compacted with ballots, which keeps both outputs in ascending slot
// order.  W = leaver sub-lists per tile (the push kernel's wavefronts per
// tile).  List slots:
//   0             : holes in [A, min(B, oA)), slots of lower old sections
//                   (hole unless the particle there moved into t)
//   1 .. W        : holes among t's W leaver sub-lists, restricted to
//                   [max(A, oA), min(B, oB))
//   W + 1         : holes in [max(A, oB), B), slots of higher old sections
//   W + 2 + q W + w : movers from the source tile of rank q (the nine tiles a
//                   particle of t can come from, ascending, duplicates
//                   dropped): s != t -- s's leaver sub-list w, entries heading
//                   to t whose slot is outside [A, B), data from the leaver
//                   records; s == t -- (w = 0, 1) t's slots outside [A, B)
//                   whose particle kept tile t
//   W + 2 + 9 W, +1 : the moving window's new particles for t outside [A, B)
// The loads are staged so that each round trip to memory serves all lists at
// once: the list bounds, then the candidates (kPlanBatch iterations of 64),
// then the movers' data, then the stores.
// candidate iterations per round trip: 6 while every tile's wavefront is
// resident at once (2048^2 in 32 x 32 tiles: each wavefront's chain of round
// trips is what counts); 2 for more tiles (a batch's tens of thousands, or
// small tiles of one large grid), which take several rounds of resident
// wavefronts, so fewer registers (more wavefronts per SIMD) count more
constexpr int kPlanBatch = 6;
constexpr int kPlanBatchB = 2;
enum : int { kListHoleRange = 0, kListHoleLeav = 1, kListMoverRange = 2, kListMoverLeav = 3 };
static_assert(10 * push_waves(32) + 4 <= 128 && 10 * push_waves(8) + 4 <= 128, "sort plan list slots");

template <int NB = kPlanBatch>
__device__ __forceinline__ void sort_plan_unit(const SortArgs &a, int spi, int grp)
{
    const int lane = threadIdx.x & 63;
    // one tile per wavefront: the index is wavefront-uniform (scalar registers)
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = grp * kSortWaves + wv;
    if (t >= a.n_tiles) return;   // whole wavefront
    const SortSpecies &sp = a.sp[spi];
    const int ntx = a.ntx, nty = a.nty;
    const int T = a.tile;
    const int W = push_waves(T);   // leaver sub-lists per tile
    const int tx = t % ntx, ty = t / ntx;
    const int gx0 = tx * T, gy0 = ty * T;

    // ---------------- the sources of t and their ranks (lanes 0..8)
    int so = -1;
    if (lane < 9) so = wrap_s(ty - (lane / 3 - 1), nty) * ntx + wrap_s(tx - (lane % 3 - 1), ntx);
    int rank = 0, first = 1;
#pragma unroll
    for (int o = 0; o < 9; ++o) {
        const int v = __shfl(so, o, 64);
        bool vfirst = true;
        for (int o2 = 0; o2 < o; ++o2)
            if (__shfl(so, o2, 64) == v) vfirst = false;
        if (vfirst && v < so) ++rank;
        if (o < lane && v == so) first = 0;
    }
    // lane o < 9: the old section of the source in offset o
    const int so_a = lane < 9 ? sp.offp[so] : 0, so_b = lane < 9 ? sp.offp[so + 1] : 0;
    // Whether the particle at `slot` of another tile's old section, with
    // tile-relative cell lc, has moved into t: its cell lies one tile off
    // its own in some offset o, and the source of t in offset o is the tile
    // whose old section holds the slot.  A particle that left the moving
    // window is in no tile.  All lanes take part.
    auto arrived = [&](int lc, int slot) {
        const int lx = tcell_x(lc), ly = tcell_y(lc);
        const int o = (ly < 0 ? 0 : (ly >= T ? 6 : 3)) + (lx < 0 ? 0 : (lx >= T ? 2 : 1));
        const int sa = __shfl(so_a, o, 64), sb = __shfl(so_b, o, 64);
        return o != 4 && (lc & 0xffff) != kTCellRemoved && slot >= sa && slot < sb;
    };
    // the source of rank q, -1 if there is none (all lanes take part)
    auto source_of_rank = [&](int q) {
        int v = -1;
#pragma unroll
        for (int o = 0; o < 9; ++o) {
            const int so_o = __shfl(so, o, 64), rank_o = __shfl(rank, o, 64), first_o = __shfl(first, o, 64);
            if (first_o && rank_o == q) v = so_o;
        }
        return v;
    };

    // ---------------- list bounds: every load of this stage in flight at once
    const int nl_mov = 9 * W;
    int srcv[2], subl[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int v = lane + 64 * h;
        const int q = v >= W + 2 && v < W + 2 + nl_mov ? (v - W - 2) / W : -1;
        subl[h] = v >= W + 2 ? (v - W - 2) % W : v - 1;   // sub-list index (movers; holes: v - 1)
        srcv[h] = source_of_rank(q);
    }
    const int A = sp.off[t], B = sp.off[t + 1];     // new section
    const int oA = sp.offp[t], oB = sp.offp[t + 1];  // old section
    int f0[2], f1[2], fc[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int v = lane + 64 * h;
        // hole sub-lists read t's record, mover sub-lists their source's (index 0 when unused)
        const int s = v >= 1 && v <= W ? t : (srcv[h] >= 0 ? srcv[h] : 0);
        const int w = v >= 1 && v <= W ? v - 1 : (srcv[h] >= 0 ? subl[h] : 0);
        f0[h] = sp.offp[s];
        f1[h] = sp.offp[s + 1];
        fc[h] = sp.cnt[(int64_t)s * kCntStride + kCntSub + w];
    }
    int i0 = 0, i1 = 0;
    if (sp.inj_off) {
        i0 = sp.n + sp.inj_off[t];
        i1 = sp.n + sp.inj_off[t + 1];
    }
    const int lA = max(A, oA), lB = min(B, oB);
    // descriptors: kind | src << 2, (base - first index), length, s0, ns
    int dks[2], dbm[2], dlen[2], ds0[2], dns[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int v = lane + 64 * h;
        int kind = kListHoleRange, base = 0, len = 0, src = 0, s0 = 0, ns = 0;
        if (v == 0) {
            base = A;
            len = max(0, min(B, oA) - A);
        } else if (v <= W) {
            int wlo, whi;
            wave_range(oA, oB, v - 1, W, wlo, whi);
            kind = kListHoleLeav;
            base = wlo;
            len = lA < lB ? min(fc[h], whi - wlo) : 0;
        } else if (v == W + 1) {
            base = max(A, oB);
            len = max(0, B - base);
        } else if (v < W + 2 + nl_mov) {
            src = srcv[h];
            const int w = subl[h];
            kind = kListMoverRange;
            if (src == t) {
                if (w == 0) {
                    base = oA;
                    len = max(0, min(oB, A) - oA);
                } else if (w == 1) {
                    base = max(oA, B);
                    len = max(0, oB - base);
                }
            } else if (src >= 0) {
                int wlo, whi;
                wave_range(f0[h], f1[h], w, W, wlo, whi);
                kind = kListMoverLeav;
                base = wlo;
                len = min(fc[h], whi - wlo);
                s0 = f0[h];
                ns = f1[h] - f0[h];
            }
            src = max(src, 0);
        } else if (v == W + 2 + nl_mov && sp.inj_off) {
            kind = kListMoverRange;
            base = i0;
            len = max(0, min(i1, A) - i0);
        } else if (v == W + 3 + nl_mov && sp.inj_off) {
            kind = kListMoverRange;
            base = max(i0, B);
            len = max(0, i1 - base);
        }
        dks[h] = kind | (src << 2);
        dbm[h] = base;
        dlen[h] = len;
        ds0[h] = s0;
        dns[h] = ns;
    }
    // the flat index space: slots 0..63 (first register), then 64..127
    int tot0, tot1;
    const int ex0 = wave_exclusive(dlen[0], tot0);
    const int ex1 = tot0 + wave_exclusive(dlen[1], tot1);
    const int total = tot0 + tot1;
    dbm[0] -= ex0;   // candidate k of the list: base + (k - ex) = dbm + k
    dbm[1] -= ex1;

    // the first slot of each pushing wavefront's run of the new section
    // (lane w < W): the holes below it give that run's first hole rank
    int wlo_mine = INT_MAX, fb = 0;
    if (lane < W) {
        int whi;
        wave_range(A, B, lane, W, wlo_mine, whi);
    }

    bool bad = false;
    int nh = 0, nm = 0;
    for (int k0 = 0; k0 < total; k0 += 64 * NB) {
        // ---- the candidates: their lists, then every load in flight at once
        int at[NB], ks[NB], s0v[NB], nsv[NB], lv[NB];
        uint32_t v[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int k = k0 + 64 * u + lane;
            const int L0 = find_list(k, ex0), L1 = find_list(k, ex1);
            const bool hi = k >= tot0;
            const int L = hi ? L1 : L0;
            auto pick = [&](const int *f) {
                const int x0 = __shfl(f[0], L, 64), x1 = __shfl(f[1], L, 64);
                return hi ? x1 : x0;
            };
            lv[u] = k < total ? L + (hi ? 64 : 0) : -1;
            ks[u] = pick(dks);
            at[u] = pick(dbm) + k;
            s0v[u] = pick(ds0);
            nsv[u] = pick(dns);
            const int kind = ks[u] & 3;
            v[u] = 0;
            if (k < total)
                v[u] = kind == kListHoleRange || kind == kListMoverRange ? (uint32_t)(int)sp.p.cell[at[u]]
                                                                         : sp.leav[at[u]];
            // a sorted state (the window's sort): every particle is in the
            // tile of its section, its cell relative to it modulo T
            if (a.rebase && (kind == kListHoleRange || kind == kListMoverRange) &&
                (v[u] & 0xffffu) != (uint32_t)kTCellRemoved)
                v[u] = (uint32_t)tcell_pack(tcell_x((int)v[u]) & (T - 1), tcell_y((int)v[u]) & (T - 1));
        }
        // ---- the ballots, in candidate order: holes first, then movers
        int rr[NB];
        unsigned mvf = 0, flf = 0;   // per iteration: a mover of this lane, from the leaver records
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int kind = ks[u] & 3, L = lv[u];
            bool ph = false, pm = false, fl = false;
            int slot = at[u];
            const bool in_t = arrived((int)v[u], slot);
            if (L >= 0) {
                if (kind == kListHoleRange) {
                    ph = !in_t;
                } else if (kind == kListHoleLeav) {
                    slot = oA + (int)(v[u] >> 4);
                    ph = slot >= lA && slot < lB;
                } else if (kind == kListMoverRange) {
                    pm = tcell_inside((int)v[u], T);   // t's own slots, or its new particles
                } else {
                    const int d = (int)(v[u] & 15u), loc = (int)(v[u] >> 4);
                    if (loc >= nsv[u] || d > kDirRemoved) {
                        bad = true;
                    } else if (d != kDirRemoved) {   // a removed particle is nobody's mover
                        const int src = ks[u] >> 2;
                        const int sx = src % ntx, sy = src / ntx;
                        const int dest = wrap_s(sy + d / 3 - 1, nty) * ntx + wrap_s(sx + d % 3 - 1, ntx);
                        const int ms = s0v[u] + loc;
                        pm = dest == t && !(ms >= A && ms < B);
                        fl = true;
                    }
                }
            }
            const unsigned long long mh = __ballot(ph);
            const int r = nh + lane_rank_s(mh);
            if (ph && r < B - A) sp.hole[(int64_t)A + r] = slot;
            nh += __popcll(mh);
            if (mh != 0ull)
                for (int w = 0; w < W; ++w) {
                    const int lo_w = __builtin_amdgcn_readlane(wlo_mine, w);
                    const int c = __popcll(__ballot(ph && slot < lo_w));
                    if (lane == w) fb += c;
                }
            const unsigned long long mm = __ballot(pm);
            rr[u] = nm + lane_rank_s(mm);
            if (pm && rr[u] < B - A) mvf |= 1u << u;
            if (fl) flf |= 1u << u;
            nm += __popcll(mm);
        }
        if (__ballot(mvf != 0) == 0ull) continue;
        // ---- the movers' data, every load in flight at once, then staged in
        // hole order (contiguous stores)
        Chunk6 dv[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u)
            if (mvf >> u & 1u) dv[u] = flf >> u & 1u ? load_leaver(sp.lrec, at[u]) : load_parts(sp.p, at[u], gx0, gy0, a.rebase ? T - 1 : -1);
#pragma unroll
        for (int u = 0; u < NB; ++u)
            if (mvf >> u & 1u) {
                const Chunk6 &c = dv[u];
                put_leaver(sp.srec, (int64_t)A + rr[u], c.cell, c.x, c.y, c.ux, c.uy, c.uz);
            }
    }

    const bool anybad = __ballot(bad) != 0ull;
    const int m = min(min(nh, nm), B - A);   // holes and movers agree unless the records were corrupt
    if (lane == 0) {
        if (nh != nm || anybad) atomicOr(a.err, kErrSort);
        sp.mcount[t] = m;
        sp.fcount[t] = a.defer ? m : 0;
    }
    if (a.defer && lane < W) sp.fbase[(int64_t)t * W + lane] = min(fb, m);
}

// Step (5): the staged movers of each tile into its holes.  Not launched
// when the sort is deferred (pic_step): the next push fills them as it
// streams the section.
__device__ __forceinline__ void sort_scatter_unit(const SortArgs &a, int spi, int grp)
{
    const int lane = threadIdx.x & 63;
    const int t = grp * kSortWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (t >= a.n_tiles) return;
    const SortSpecies &sp = a.sp[spi];
    const int A = sp.off[t], m = sp.mcount[t];
    const int gx0 = (t % a.ntx) * a.tile, gy0 = (t / a.ntx) * a.tile;
    for (int k = lane; k < m; k += 64) {
        const int64_t r = (int64_t)A + k;
        store_parts(sp.p, sp.hole[r], load_leaver(sp.srec, r), gx0, gy0);
    }
}

// ---- The motion-class sort (the alternative of Sec. 4.3, after
// Germaschewski et al.): by the Courant condition a particle ends a step in
// its own tile or one of the eight around it, so its motion falls into one of
// nine classes d = (dty + 1) * 3 + (dtx + 1) -- the step from the tile whose
// section holds it to its new tile, counted +1 on an axis of two tiles, the
// push kernel's direction code -- and the push has already counted the
// particles of every (tile, class).  One pass then moves every particle of
// source tile s and class d to its place in the new order (new tile, class,
// old slot) in the staging arrays: base(s, d) = the new section start of the
// destination tile t = s + step(d), plus the counts of the classes before d
// arriving at t from their own source tiles.  A second pass copies the
// staging arrays back.  Out of place: reads and writes every particle twice,
// so it pays only when most particles change tile.

// The motion class of a particle with tile-relative cell lc (tiles of edge
// T, ntx x nty of them): the push kernel's direction code of the step to the
// tile it is in now (+1 on an axis of two tiles, either way), or 9 if that
// is more than one tile away or the particle left the moving window.
__device__ __forceinline__ int motion_class(int lc, int T, int ntx, int nty)
{
    const int lx = tcell_x(lc), ly = tcell_y(lc);
    const int stx = lx < 0 ? (ntx == 2 ? 1 : -1) : (lx >= T ? 1 : 0);
    const int sty = ly < 0 ? (nty == 2 ? 1 : -1) : (ly >= T ? 1 : 0);
    const bool far = lx < -T || lx >= 2 * T || ly < -T || ly >= 2 * T;   // the removed mark too
    return far ? 9 : (sty + 1) * 3 + (stx + 1);
}

struct Part6 {
    int cell;
    float x, y, ux, uy, uz;
};

// A whole-array pass of the motion-class sort reads every particle once, so
// its loads carry the non-temporal hint (as the push's particle stream
// does); its stores start mid-line (class runs), where the hint costs.
__device__ __forceinline__ Part6 load_part(const Parts &p, int i)
{
    return Part6{__builtin_nontemporal_load(p.cell + i), __builtin_nontemporal_load(p.x + i),
                 __builtin_nontemporal_load(p.y + i),    __builtin_nontemporal_load(p.ux + i),
                 __builtin_nontemporal_load(p.uy + i),   __builtin_nontemporal_load(p.uz + i)};
}

__device__ __forceinline__ void store_part(const Parts &p, int i, const Part6 &v)
{
    p.cell[i] = v.cell;
    p.x[i] = v.x;
    p.y[i] = v.y;
    p.ux[i] = v.ux;
    p.uy[i] = v.uy;
    p.uz[i] = v.uz;
}

// The nt source tiles from tile t0 on, one after the other, each by the whole
// block: the section's 64-aligned chunks are split into one run per
// wavefront; a first pass counts every run's particles per class, a second
// streams the runs again and moves each particle to its slot (its class's
// first slot in the destination, the class's particles in the earlier runs,
// its rank in its chunk).  One tile per block for a single simulation (many
// wavefronts in flight), kSortWaves per work item in a batch.
__device__ __forceinline__ void motion_scatter_unit(const SortArgs &a, int spi, int t0, int nt)
{
    constexpr int W = kSortWaves;
    __shared__ int s_cls[W][9];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const SortSpecies &sp = a.sp[spi];
    const int ntx = a.ntx, nty = a.nty;
    const int T = a.tile;
    for (int q = 0; q < nt; ++q) {
        const int s = t0 + q;
        if (s >= a.n_tiles) break;   // uniform over the block
        const int sx = s % ntx, sy = s / ntx;
        const int oA = sp.offp[s], oB = sp.offp[s + 1];
        int lo, hi;
        wave_range(oA, oB, w, W, lo, hi);
        // pass 1: lane d counts the run's particles of class d
        int mine = 0;
        for (int c0 = (lo >> 6) << 6; c0 < hi; c0 += 64) {
            const int i = c0 + lane;
            const int d = (i >= lo && i < hi) ? motion_class(sp.p.cell[i], T, ntx, nty) : 10;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const int c = __popcll(__ballot(d == k));
                if (lane == k) mine += c;
            }
        }
        if (lane < 9) s_cls[w][lane] = mine;
        __syncthreads();
        // lane d < 9: the run's first slot for class d and the class's end
        int pos = 0, end = 0;
        bool bad = false;
        if (lane < 9) {
            const int dx = lane % 3 - 1, dy = lane / 3 - 1;
            const int t = wrap_s(sy + dy, nty) * ntx + wrap_s(sx + dx, ntx);
            const int tx = t % ntx, ty = t / ntx;
            pos = sp.off[t];
            for (int d2 = 0; d2 < lane; ++d2) {
                const int src = wrap_s(ty - (d2 / 3 - 1), nty) * ntx + wrap_s(tx - (d2 % 3 - 1), ntx);
                pos += sp.cnt[(int64_t)src * kCntStride + d2];
            }
            const int total = sp.cnt[(int64_t)s * kCntStride + lane];
            end = pos + total;
            int all = 0;
            for (int w2 = 0; w2 < W; ++w2) {
                if (w2 < w) pos += s_cls[w2][lane];
                all += s_cls[w2][lane];
            }
            bad = all != total;   // the push's counts and the cells disagree
        }
        // pass 2: the particles to their slots, the next two chunks in flight
        int c0 = (lo >> 6) << 6;
        Part6 nxt{}, nxt2{};
        if (c0 + lane >= lo && c0 + lane < hi) nxt = load_part(sp.p, c0 + lane);
        if (c0 + 64 + lane >= lo && c0 + 64 + lane < hi) nxt2 = load_part(sp.p, c0 + 64 + lane);
        for (; c0 < hi; c0 += 64) {
            const Part6 cur = nxt;
            nxt = nxt2;
            const int i = c0 + lane;
            const bool in = i >= lo && i < hi;
            const int i3 = i + 128;
            if (i3 >= lo && i3 < hi) nxt2 = load_part(sp.p, i3);
            const int d = in ? motion_class(cur.cell, T, ntx, nty) : 10;
            unsigned long long m_d = 0ull;
            int taken = 0;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const unsigned long long m = __ballot(d == k);
                if (d == k) m_d = m;
                if (lane == k) taken = __popcll(m);
            }
            const int at = __shfl(pos, d < 9 ? d : 0, 64) + lane_rank_s(m_d);
            const int lim = __shfl(end, d < 9 ? d : 0, 64);
            if (in) {
                if (d < 9 && at < lim && (unsigned)at < (unsigned)sp.n) {
                    Part6 v = cur;   // its cell relative to the tile it is in now
                    v.cell = tcell_pack(tcell_x(cur.cell) & (T - 1), tcell_y(cur.cell) & (T - 1));
                    store_part(sp.stg, at, v);
                }
                else bad = true;
            }
            pos += taken;
        }
        const bool anybad = __ballot(bad) != 0ull;
        if (lane == 0 && anybad) atomicOr(a.err, kErrSort);
        if (threadIdx.x == 0) sp.mcount[s] = 0;   // pic_diag's mover count: not tracked by this sort
        __syncthreads();   // s_cls is reused by the next tile
    }
    // the copy back is left to the next push (read by launches after this one)
    if (a.defer && threadIdx.x == 0) *a.stg_live = 1;
}

// The new sections of the nt tiles from t0 on (contiguous) from the staging
// arrays into the particle arrays, by the whole block, four particles per
// thread in flight; live: only if the copy was left pending (*stg_live).
__device__ __forceinline__ void motion_copy_unit(const SortArgs &a, int spi, int t0, int nt, bool live = false)
{
    if (live && *a.stg_live == 0) return;
    const SortSpecies &sp = a.sp[spi];
    if (t0 >= a.n_tiles) return;
    const int t1 = min(t0 + nt, a.n_tiles);
    const int A = sp.off[t0], B = sp.off[t1];
    constexpr int U = 4;
    for (int i0 = A + (int)threadIdx.x; i0 < B; i0 += U * kBlock) {
        Part6 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i0 + u * kBlock < B) v[u] = load_part(sp.stg, i0 + u * kBlock);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i0 + u * kBlock < B) store_part(sp.p, i0 + u * kBlock, v[u]);
    }
}

// ---- single-simulation kernels: blockIdx.y = species
__global__ void __launch_bounds__(kScanBlock) k_sort_count(SortArgs a) { sort_count_unit(a, blockIdx.y, blockIdx.x); }
__global__ void __launch_bounds__(1024) k_sort_scan_blocks(SortArgs a) { sort_scan_unit(a, blockIdx.x); }
__global__ void __launch_bounds__(kScanBlock) k_sort_add_base(SortArgs a) { sort_add_unit(a, blockIdx.y, blockIdx.x); }
__global__ void __launch_bounds__(kScanBlock) k_sort_add_direct(SortArgs a)
{
    sort_add_direct_unit(a, blockIdx.y, blockIdx.x);
}
// A fill left pending by a deferred sort, done on its own (before anything
// reads the particle arrays other than a push): tile t's fcount[t] staged
// movers into its holes, as the next push would, and fcount[t] back to 0.
__device__ __forceinline__ void fill_unit(const SortArgs &a, int spi, int grp)
{
    const int lane = threadIdx.x & 63;
    const int t = grp * kSortWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (t >= a.n_tiles) return;
    const SortSpecies &sp = a.sp[spi];
    const int A = sp.off[t], m = sp.fcount[t];
    const int gx0 = (t % a.ntx) * a.tile, gy0 = (t / a.ntx) * a.tile;
    for (int k = lane; k < m; k += 64) {
        const int64_t r = (int64_t)A + k;
        store_parts(sp.p, sp.hole[r], load_leaver(sp.srec, r), gx0, gy0);
    }
    if (lane == 0 && m != 0) sp.fcount[t] = 0;
}

// The whole-grid cells of tile t's section into the caller's cell array
// (one wavefront per tile), from the tile-relative ones: the cell of a
// particle that has left its tile wraps across the periodic seam.  rebase:
// a sorted state, each cell relative to the tile modulo its edge.
__device__ __forceinline__ void publish_unit(const SortArgs &a, int spi, int grp, bool rebase)
{
    const int lane = threadIdx.x & 63;
    const int t = grp * kSortWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (t >= a.n_tiles) return;
    const SortSpecies &sp = a.sp[spi];
    const int gx0 = (t % a.ntx) * a.tile, gy0 = (t / a.ntx) * a.tile;
    const int A = sp.off[t], B = sp.off[t + 1];
    const int mask = rebase ? a.tile - 1 : -1;
    for (int i = A + lane; i < B; i += 64) {
        const int lc = sp.p.cell[i];
        sp.gcell[i] = wrap_s(gx0 + (tcell_x(lc) & mask), a.nx) | (wrap_s(gy0 + (tcell_y(lc) & mask), a.ny) << 16);
    }
}

__global__ void __launch_bounds__(kBlock) k_fill(SortArgs a) { fill_unit(a, blockIdx.y, blockIdx.x); }
__global__ void __launch_bounds__(kBlock) k_publish(SortArgs a, int rebase)
{
    publish_unit(a, blockIdx.y, blockIdx.x, rebase != 0);
}
template <int NB>
__global__ void __launch_bounds__(kBlock) k_sort_plan(SortArgs a) { sort_plan_unit<NB>(a, blockIdx.y, blockIdx.x); }
__global__ void __launch_bounds__(kBlock) k_sort_scatter(SortArgs a) { sort_scatter_unit(a, blockIdx.y, blockIdx.x); }
// single simulation: one tile per block
__global__ void __launch_bounds__(kBlock) k_motion_scatter(SortArgs a) { motion_scatter_unit(a, blockIdx.y, blockIdx.x, 1); }
__global__ void __launch_bounds__(kBlock) k_motion_copy(SortArgs a) { motion_copy_unit(a, blockIdx.y, blockIdx.x, 1); }
__global__ void __launch_bounds__(kBlock) k_motion_copy_live(SortArgs a)
{
    motion_copy_unit(a, blockIdx.y, blockIdx.x, 1, true);
}

// ---- many simulations: one block per work item (sim, species, unit)
__global__ void __launch_bounds__(kScanBlock) k_sort_count_b(const SortArgs *d, const int4 *it)
{
    const int4 w = it[blockIdx.x];
    sort_count_unit(d[w.x], w.y, w.z);
}
__global__ void __launch_bounds__(1024) k_sort_scan_blocks_b(const SortArgs *d, const int4 *it)
{
    const int4 w = it[blockIdx.x];
    sort_scan_unit(d[w.x], w.y);
}
__global__ void __launch_bounds__(kScanBlock) k_sort_add_direct_b(const SortArgs *d, const int4 *it)
{
    const int4 w = it[blockIdx.x];
    sort_add_direct_unit(d[w.x], w.y, w.z);
}
__global__ void __launch_bounds__(kScanBlock) k_sort_add_base_b(const SortArgs *d, const int4 *it)
{
    const int4 w = it[blockIdx.x];
    sort_add_unit(d[w.x], w.y, w.z);
}
__global__ void __launch_bounds__(kBlock) k_sort_plan_b(const SortArgs *d, const int4 *it)
{
    const int4 w = it[blockIdx.x];
    sort_plan_unit<kPlanBatchB>(d[w.x], w.y, w.z);
}
__global__ void __launch_bounds__(kBlock) k_fill_b(const SortArgs *d, const int4 *it)
{
    const int4 w = it[blockIdx.x];
    fill_unit(d[w.x], w.y, w.z);
}
__global__ void __launch_bounds__(kBlock) k_publish_b(const SortArgs *d, const int4 *it, int rebase)
{
    const int4 w = it[blockIdx.x];
    publish_unit(d[w.x], w.y, w.z, rebase != 0);
}

__global__ void __launch_bounds__(kBlock) k_motion_scatter_b(const SortArgs *d, const int4 *it)
{
    const int4 w = it[blockIdx.x];
    motion_scatter_unit(d[w.x], w.y, w.z * kSortWaves, kSortWaves);
}
__global__ void __launch_bounds__(kBlock) k_motion_copy_b(const SortArgs *d, const int4 *it)
{
    const int4 w = it[blockIdx.x];
    motion_copy_unit(d[w.x], w.y, w.z * kSortWaves, kSortWaves);
}

// ---- tile_offset from caller particles: whether every cell is in the grid
// (kErrOrder) and the cells are grouped by tile (kErrGroup), then, for
// grouped cells, off[t] = the first slot whose tile is >= t (a binary search
// per tile: no atomics, so many particles per tile cost nothing extra)
__global__ void k_init_check(const int32_t *__restrict__ cell, int32_t n, int nx, int ny, int tsh, int ntx,
                             int *err)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = cell[i];
    const int ix = c & 0xffff, iy = c >> 16;
    if (c < 0 || ix >= nx || iy >= ny) {
        atomicOr(err, kErrOrder);
        return;
    }
    if (i + 1 < n) {
        const int c2 = cell[i + 1];
        const int t = (iy >> tsh) * ntx + (ix >> tsh);
        const int t2 = ((c2 >> 16) >> tsh) * ntx + ((c2 & 0xffff) >> tsh);
        if (c2 >= 0 && t2 < t) atomicOr(err, kErrGroup);
    }
}

__global__ void k_init_offsets(const int32_t *__restrict__ cell, int32_t n, int tsh, int ntx, int n_tiles,
                               int32_t *__restrict__ off)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t > n_tiles) return;
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = lo + ((hi - lo) >> 1);
        const int c = cell[mid];
        const int tm = c < 0 ? -1 : ((c >> 16) >> tsh) * ntx + ((c & 0xffff) >> tsh);
        if (tm < t) lo = mid + 1;
        else hi = mid;
    }
    off[t] = lo;
}

void launch_sort_scan(const SortArgs &a, int n_tiles, hipStream_t s)
{
    const int nb = (n_tiles + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(k_sort_count, dim3(nb, a.n_species), dim3(kScanBlock), 0, s, a);
    if (nb <= kScanDirect) {
        hipLaunchKernelGGL(k_sort_add_direct, dim3(nb, a.n_species), dim3(kScanBlock), 0, s, a);
        return;
    }
    hipLaunchKernelGGL(k_sort_scan_blocks, dim3(a.n_species), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_sort_add_base, dim3(nb, a.n_species), dim3(kScanBlock), 0, s, a);
}

// Plan wavefronts (one per tile and species) that fit the device at once with
// the six-iteration plan (four wavefronts per SIMD, 256 CUs); beyond, the
// two-iteration plan runs twice as many at once.
constexpr int64_t kPlanResident = 4096;

void launch_sort_plan(const SortArgs &a, int n_tiles, hipStream_t s)
{
    const dim3 grid((n_tiles + kSortWaves - 1) / kSortWaves, a.n_species);
    if ((int64_t)n_tiles * a.n_species <= kPlanResident)
        hipLaunchKernelGGL(k_sort_plan<kPlanBatch>, grid, dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_sort_plan<kPlanBatchB>, grid, dim3(kBlock), 0, s, a);
}

void launch_sort_scatter(const SortArgs &a, int n_tiles, hipStream_t s)
{
    hipLaunchKernelGGL(k_sort_scatter, dim3((n_tiles + kSortWaves - 1) / kSortWaves, a.n_species), dim3(kBlock), 0,
                       s, a);
}

void launch_fill(const SortArgs &a, int n_tiles, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, dim3((n_tiles + kSortWaves - 1) / kSortWaves, a.n_species), dim3(kBlock), 0, s, a);
}

void launch_fill_batch(const SortBatch &b, hipStream_t s)
{
    if (b.n_plan > 0) hipLaunchKernelGGL(k_fill_b, dim3(b.n_plan), dim3(kBlock), 0, s, b.descs, b.plan_items);
}

void launch_publish(const SortArgs &a, int n_tiles, bool rebase, hipStream_t s)
{
    hipLaunchKernelGGL(k_publish, dim3((n_tiles + kSortWaves - 1) / kSortWaves, a.n_species), dim3(kBlock), 0, s, a,
                       rebase ? 1 : 0);
}

void launch_publish_batch(const SortBatch &b, bool rebase, hipStream_t s)
{
    if (b.n_plan > 0)
        hipLaunchKernelGGL(k_publish_b, dim3(b.n_plan), dim3(kBlock), 0, s, b.descs, b.plan_items, rebase ? 1 : 0);
}

void launch_sort_batch(const SortBatch &b, bool motion, hipStream_t s)
{
    if (b.n_count == 0) return;
    hipLaunchKernelGGL(k_sort_count_b, dim3(b.n_count), dim3(kScanBlock), 0, s, b.descs, b.count_items);
    if (b.max_blocks <= kScanDirect) {
        hipLaunchKernelGGL(k_sort_add_direct_b, dim3(b.n_count), dim3(kScanBlock), 0, s, b.descs, b.count_items);
    } else {
        hipLaunchKernelGGL(k_sort_scan_blocks_b, dim3(b.n_scan), dim3(1024), 0, s, b.descs, b.scan_items);
        hipLaunchKernelGGL(k_sort_add_base_b, dim3(b.n_count), dim3(kScanBlock), 0, s, b.descs, b.count_items);
    }
    if (motion) {
        hipLaunchKernelGGL(k_motion_scatter_b, dim3(b.n_plan), dim3(kBlock), 0, s, b.descs, b.plan_items);
        hipLaunchKernelGGL(k_motion_copy_b, dim3(b.n_plan), dim3(kBlock), 0, s, b.descs, b.plan_items);
    } else {
        // the batched in-place sort is deferred: the next batched push fills the holes
        hipLaunchKernelGGL(k_sort_plan_b, dim3(b.n_plan), dim3(kBlock), 0, s, b.descs, b.plan_items);
    }
}

void launch_motion_scatter(const SortArgs &a, int n_tiles, hipStream_t s)
{
    hipLaunchKernelGGL(k_motion_scatter, dim3(n_tiles, a.n_species), dim3(kBlock), 0, s, a);
}

void launch_motion_copy(const SortArgs &a, int n_tiles, hipStream_t s)
{
    hipLaunchKernelGGL(k_motion_copy, dim3(n_tiles, a.n_species), dim3(kBlock), 0, s, a);
}

void launch_motion_copy_live(const SortArgs &a, int n_tiles, hipStream_t s)
{
    hipLaunchKernelGGL(k_motion_copy_live, dim3(n_tiles, a.n_species), dim3(kBlock), 0, s, a);
    launch_set_int(a.stg_live, 0, s);
}

// Tile-relative cells of n particles grouped by tile, each inside its tile
// (checked before), from their whole-grid cells.
__global__ void __launch_bounds__(256) k_localize(const int32_t *__restrict__ cell, int16_t *__restrict__ lcell,
                                                  int32_t n, int tile)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = cell[i];
    lcell[i] = (int16_t)tcell_pack((c & 0xffff) & (tile - 1), (c >> 16) & (tile - 1));
}

void launch_localize(const int32_t *cell, int16_t *lcell, int32_t n, int tile, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_localize, dim3((n + 255) / 256), dim3(256), 0, s, cell, lcell, n, tile);
}

void launch_init_tiles(const int32_t *cell, int32_t n, int nx, int ny, int tile, int ntx, int n_tiles, int32_t *off,
                       int *err, hipStream_t s)
{
    const int tsh = __builtin_ctz(tile);
    if (n > 0)
        hipLaunchKernelGGL(k_init_check, dim3((n + 255) / 256), dim3(256), 0, s, cell, n, nx, ny, tsh, ntx, err);
    hipLaunchKernelGGL(k_init_offsets, dim3((n_tiles + 1 + 255) / 256), dim3(256), 0, s, cell, n, tsh, ntx, n_tiles,
                       off);
}

}  // namespace pic

// Strict re-sort of particles by tile (Sec. 4.3, the bucket sort of Fig. 4.5),
// redesigned for gfx950: no atomics decide any position, so the permutation
// is the canonical one and is reproducible bit for bit.
//
//   k_sort_scan    step (1): the new count of tile t is the sum, over the nine
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
//                  the movers are gathered into a staging area at once, so
//                  only O(movers) particle bytes are touched.
//   k_sort_scatter step (5): the k-th hole receives the k-th mover.
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

__global__ void __launch_bounds__(1024) k_sort_scan(SortArgs a, int n_tiles)
{
    const SortSpecies &sp = a.sp[blockIdx.x];
    const int per = (n_tiles + 1023) / 1024;
    const int t0 = min((int)threadIdx.x * per, n_tiles), t1 = min(t0 + per, n_tiles);
    int sum = 0;
    for (int t = t0; t < t1; ++t) sum += tile_count_in(sp.cnt, t, a.ntx, a.nty);
    int total;
    int base = block_exclusive_scan_1024(sum, &total);
    for (int t = t0; t < t1; ++t) {
        sp.offn[t] = base;
        base += tile_count_in(sp.cnt, t, a.ntx, a.nty);
    }
    if (threadIdx.x == 0) {
        sp.offn[n_tiles] = total;
        if (total != sp.n) atomicOr(a.err, kErrCount);
    }
}

__global__ void __launch_bounds__(kBlock) k_sort_plan(SortArgs a, int n_tiles)
{
    const int lane = threadIdx.x & 63;
    const int t = blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (t >= n_tiles) return;   // whole wavefront
    const SortSpecies &sp = a.sp[blockIdx.y];
    const int ntx = a.ntx, nty = a.nty;
    const int tsh = __builtin_ctz(a.tile);
    const int A = sp.offn[t], B = sp.offn[t + 1];
    const int oA = sp.off[t], oB = sp.off[t + 1];

    auto tile_of = [&](int cell) { return ((cell >> 16) >> tsh) * ntx + ((cell & 0xffff) >> tsh); };

    // ---------------- holes, ascending
    int nh = 0;
    auto hole_scan = [&](int lo, int hi, bool want_foreign) {
        for (int b = lo; b < hi; b += 64) {
            const int i = b + lane;
            bool p = false;
            if (i < hi) p = (tile_of(sp.cell[i]) != t) == want_foreign;
            const unsigned long long m = __ballot(p);
            if (p && nh + lane_rank_s(m) < B - A) sp.hole[(int64_t)A + nh + lane_rank_s(m)] = i;
            nh += __popcll(m);
        }
    };
    // part of [A, B) below t's old section: holes unless the particle moved into t
    hole_scan(A, min(B, oA), true);
    // part of [A, B) inside t's old section: holes are t's leavers there
    {
        const int lA = max(A, oA), lB = min(B, oB);
        if (lA < lB) {
            for (int w = 0; w < kWaves; ++w) {
                const int cw = sp.cnt[(int64_t)t * kCntStride + kCntSub + w];
                int wlo, whi;
                wave_range(oA, oB, w, wlo, whi);
                const int64_t base = wlo;
                for (int b = 0; b < cw; b += 64) {
                    const int k = b + lane;
                    bool p = false;
                    int slot = 0;
                    if (k < cw && k < whi - wlo) {
                        slot = oA + (int)(sp.leav[base + k] >> 4);
                        p = slot >= lA && slot < lB;
                    }
                    const unsigned long long m = __ballot(p);
                    if (p && nh + lane_rank_s(m) < B - A) sp.hole[(int64_t)A + nh + lane_rank_s(m)] = slot;
                    nh += __popcll(m);
                }
            }
        }
    }
    // part of [A, B) above t's old section
    hole_scan(max(A, oB), B, true);

    // ---------------- movers, ascending old slot, gathered into staging
    int nm = 0;
    bool bad = false;
    auto gather = [&](bool p, int slot) {
        const unsigned long long m = __ballot(p);
        if (p) {
            const int r = A + nm + lane_rank_s(m);
            if (r < B) {
                sp.stg_cell[r] = sp.cell[slot];
                sp.stg_x[r] = sp.x[slot];
                sp.stg_y[r] = sp.y[slot];
                sp.stg_ux[r] = sp.ux[slot];
                sp.stg_uy[r] = sp.uy[slot];
                sp.stg_uz[r] = sp.uz[slot];
            }
        }
        nm += __popcll(m);
    };

    // the nine tiles a particle of t can come from, ascending, duplicates dropped
    const int tx = t % ntx, ty = t / ntx;
    int src[9];
#pragma unroll
    for (int o = 0; o < 9; ++o) src[o] = wrap_s(ty - (o / 3 - 1), nty) * ntx + wrap_s(tx - (o % 3 - 1), ntx);
#pragma unroll
    for (int i = 1; i < 9; ++i)
#pragma unroll
        for (int j = i; j > 0; --j)
            if (src[j] < src[j - 1]) {
                const int tmp = src[j];
                src[j] = src[j - 1];
                src[j - 1] = tmp;
            }

#pragma unroll
    for (int o = 0; o < 9; ++o) {
        const int s = src[o];
        if (o > 0 && s == src[o - 1]) continue;
        if (s == t) {
            // t's own particles outside [A, B) that kept tile t
            const int lo1 = oA, hi1 = min(oB, A), lo2 = max(oA, B), hi2 = oB;
            for (int r = 0; r < 2; ++r) {
                const int lo = r ? lo2 : lo1, hi = r ? hi2 : hi1;
                for (int b = lo; b < hi; b += 64) {
                    const int i = b + lane;
                    const bool p = i < hi && tile_of(sp.cell[i]) == t;
                    gather(p, i);
                }
            }
        } else {
            const int so = sp.off[s], ns = sp.off[s + 1] - so;
            const int sx = s % ntx, sy = s / ntx;
            for (int w = 0; w < kWaves; ++w) {
                const int cw = sp.cnt[(int64_t)s * kCntStride + kCntSub + w];
                int wlo, whi;
                wave_range(so, so + ns, w, wlo, whi);
                const int64_t base = wlo;
                for (int b = 0; b < cw; b += 64) {
                    const int k = b + lane;
                    bool p = false;
                    int slot = 0;
                    if (k < cw && k < whi - wlo) {
                        const uint32_t e = sp.leav[base + k];
                        const int d = (int)(e & 15u), loc = (int)(e >> 4);
                        const int dest = wrap_s(sy + d / 3 - 1, nty) * ntx + wrap_s(sx + d % 3 - 1, ntx);
                        if (loc >= ns || d > 8) {
                            bad = true;
                        } else {
                            slot = so + loc;
                            p = dest == t && !(slot >= A && slot < B);
                        }
                    }
                    gather(p, slot);
                }
            }
        }
    }

    if (lane == 0) {
        if (nh != nm || bad) atomicOr(a.err, kErrSort);
        sp.mcount[t] = min(nh, nm);
    }
    if (__ballot(bad) != 0ull && lane == 0) atomicOr(a.err, kErrSort);
}

__global__ void __launch_bounds__(kBlock) k_sort_scatter(SortArgs a, int n_tiles)
{
    const int lane = threadIdx.x & 63;
    const int t = blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (t >= n_tiles) return;
    const SortSpecies &sp = a.sp[blockIdx.y];
    const int A = sp.offn[t], m = sp.mcount[t];
    for (int k = lane; k < m; k += 64) {
        const int64_t r = (int64_t)A + k;
        const int dst = sp.hole[r];
        sp.cell[dst] = sp.stg_cell[r];
        sp.x[dst] = sp.stg_x[r];
        sp.y[dst] = sp.stg_y[r];
        sp.ux[dst] = sp.stg_ux[r];
        sp.uy[dst] = sp.stg_uy[r];
        sp.uz[dst] = sp.stg_uz[r];
    }
}

// ---- initial tile_offset from caller particles that are grouped by tile
__global__ void k_init_count(const int32_t *__restrict__ cell, int32_t n, int nx, int ny, int tsh,
                             int ntx, int32_t *counts, int *err)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = cell[i];
    const int ix = c & 0xffff, iy = c >> 16;
    if (c < 0 || ix >= nx || iy >= ny) {
        atomicOr(err, kErrOrder);
        return;
    }
    const int t = (iy >> tsh) * ntx + (ix >> tsh);
    atomicAdd(&counts[t], 1);
    if (i + 1 < n) {
        const int c2 = cell[i + 1];
        const int t2 = ((c2 >> 16) >> tsh) * ntx + ((c2 & 0xffff) >> tsh);
        if (c2 >= 0 && t2 < t) atomicOr(err, kErrOrder);
    }
}

__global__ void __launch_bounds__(1024) k_init_scan(const int32_t *counts, int n_tiles, int32_t *off,
                                                     int32_t n, int *err)
{
    const int per = (n_tiles + 1023) / 1024;
    const int t0 = min((int)threadIdx.x * per, n_tiles), t1 = min(t0 + per, n_tiles);
    int sum = 0;
    for (int t = t0; t < t1; ++t) sum += counts[t];
    int total;
    int base = block_exclusive_scan_1024(sum, &total);
    for (int t = t0; t < t1; ++t) {
        off[t] = base;
        base += counts[t];
    }
    if (threadIdx.x == 0) {
        off[n_tiles] = total;
        if (total != n) atomicOr(err, kErrOrder);
    }
}

void launch_sort_scan(const SortArgs &a, int n_tiles, hipStream_t s)
{
    hipLaunchKernelGGL(k_sort_scan, dim3(a.n_species), dim3(1024), 0, s, a, n_tiles);
}

void launch_sort_plan(const SortArgs &a, int n_tiles, hipStream_t s)
{
    hipLaunchKernelGGL(k_sort_plan, dim3((n_tiles + kWaves - 1) / kWaves, a.n_species), dim3(kBlock), 0, s,
                       a, n_tiles);
}

void launch_sort_scatter(const SortArgs &a, int n_tiles, hipStream_t s)
{
    hipLaunchKernelGGL(k_sort_scatter, dim3((n_tiles + kWaves - 1) / kWaves, a.n_species), dim3(kBlock), 0,
                       s, a, n_tiles);
}

void launch_init_tiles(const int32_t *cell, int32_t n, int nx, int ny, int tile, int ntx, int32_t *counts,
                       int n_tiles, int32_t *off, int *err, hipStream_t s)
{
    const int tsh = __builtin_ctz(tile);
    if (n > 0)
        hipLaunchKernelGGL(k_init_count, dim3((n + 255) / 256), dim3(256), 0, s, cell, n, nx, ny, tsh, ntx,
                           counts, err);
    hipLaunchKernelGGL(k_init_scan, dim3(1), dim3(1024), 0, s, counts, n_tiles, off, n, err);
}

}  // namespace pic

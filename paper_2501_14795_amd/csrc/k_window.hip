// The moving-window step at the end of Listing 3.1.  The grid is periodic
// between window moves, so moving every field value and every particle one
// cell towards -x is a relabelling of the array columns: window column i is
// kept in array column (i + origin) mod nx, and a move advances the origin by
// one.  What remains to do is local to one array column `col` (window column
// 0 before the move, window column nx - 1 after it): E and B there become
// zero, its particles leave, and the new particles come in there.  The
// particle half emits exactly what the push kernel emits for the sort --
// per-wavefront leaver sub-lists in slot order and count records -- so the
// same canonical sort closes the holes and places the new particles.
#include "pic_internal.h"

namespace pic {

// E and B (planes 0..5) of array column `col` become zero
__global__ void __launch_bounds__(256) k_zero_column(float *__restrict__ fld, int nx, int ny, int col)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ny) return;
    const int64_t P = (int64_t)nx * ny;
    const int64_t k = (int64_t)j * nx + col;
    for (int c = 0; c < 6; ++c) fld[c * P + k] = 0.0f;
}

// Count records of a step in which nothing moves: all particles of a tile
// stay (direction 4), no leavers.  One thread per record entry.
__global__ void __launch_bounds__(256) k_window_records(const int32_t *__restrict__ off, int32_t *__restrict__ cnt,
                                                        int n_tiles)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_tiles * kCntStride) return;
    const int t = (int)(i / kCntStride), k = (int)(i % kCntStride);
    cnt[i] = k == 4 ? off[t + 1] - off[t] : 0;
}

// The tiles of the tile column that holds array column `col`, one per
// workgroup of push_waves(T) wavefronts, each streaming the run of the
// section the push kernel would give it.  A particle in column `col` leaves
// (its cell marked kTCellRemoved, direction kDirRemoved); every other
// particle stays.  The particles are sorted: each lies in its own tile.
template <int T>
__global__ void __launch_bounds__(64 * push_waves(T)) k_window_remove(WindowSpecies w, int ntx, int col)
{
    constexpr int W = push_waves(T);
    __shared__ int s_wl[W];
    const int tile = blockIdx.x * ntx + col / T;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int begin = w.off[tile], end = w.off[tile + 1];
    int lo, hi;
    wave_range(begin, end, wave, W, lo, hi);
    int nleav = 0;   // wavefront-uniform
    for (int cb = (lo >> 6) << 6; cb < hi; cb += 64) {
        const int i = cb + lane;
        bool leaves = false;
        if (i >= lo && i < hi) {
            // sorted: the cell is relative to the tile modulo T
            leaves = (tcell_x(w.p.cell[i]) & (T - 1)) == (col & (T - 1));
            if (leaves) w.p.cell[i] = (int16_t)kTCellRemoved;
        }
        const unsigned long long m = __ballot(leaves);
        if (leaves) {
            const int64_t q = (int64_t)lo + nleav + (int)__builtin_amdgcn_mbcnt_hi(
                                  (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            w.leav[q] = ((uint32_t)(i - begin) << 4) | (uint32_t)kDirRemoved;
        }
        nleav += __popcll(m);
    }
    if (lane == 0) s_wl[wave] = nleav;
    __syncthreads();
    if (threadIdx.x < kCntStride) {
        const int k = threadIdx.x;
        int leavers = 0;
        for (int q = 0; q < W; ++q) leavers += s_wl[q];
        int v = 0;
        if (k == 4) v = (end - begin) - leavers;
        else if (k == kCntLeavers) v = leavers;
        else if (k >= kCntSub && k < kCntSub + W) v = s_wl[k - kCntSub];
        w.cnt[(int64_t)tile * kCntStride + k] = v;
        if (k == 0 && leavers) atomicAdd(w.removed, leavers);
    }
}

// The new particles, given in window column nx - 1, into array column `col`:
// dst[i] = col | iy << 16 and, relative to their tile, ldst[i].  Anything
// else sets kErrOrder (and is written clamped into the grid, so later kernels
// of the same call stay in bounds).
__global__ void __launch_bounds__(256) k_place_new(const int32_t *__restrict__ src, int32_t *__restrict__ dst,
                                                   int16_t *__restrict__ ldst, int n, int nx, int ny, int col,
                                                   int tile, int *err)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = src[i];
    const int ix = c & 0xffff, iy = c >> 16;
    const bool ok = c >= 0 && ix == nx - 1 && iy < ny;
    if (!ok) atomicOr(err, kErrOrder);
    const int jy = ok ? iy : 0;
    dst[i] = col | (jy << 16);
    ldst[i] = (int16_t)tcell_pack(col & (tile - 1), jy & (tile - 1));
}

__global__ void __launch_bounds__(256) k_zero_i32(int32_t *__restrict__ p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

void launch_zero_i32(int32_t *p, int n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_zero_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
}

void launch_zero_column(float *fld, int nx, int ny, int col, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_column, dim3((ny + 255) / 256), dim3(256), 0, s, fld, nx, ny, col);
}

void launch_window_remove(int tile, const WindowSpecies &w, int ntx, int nty, int n_tiles, int col, hipStream_t s)
{
    if (n_tiles <= 0) return;
    const int64_t entries = (int64_t)n_tiles * kCntStride;
    hipLaunchKernelGGL(k_window_records, dim3((unsigned)((entries + 255) / 256)), dim3(256), 0, s, w.off, w.cnt,
                       n_tiles);
    switch (tile) {
    case 8: hipLaunchKernelGGL((k_window_remove<8>), dim3(nty), dim3(64 * push_waves(8)), 0, s, w, ntx, col); break;
    case 16:
        hipLaunchKernelGGL((k_window_remove<16>), dim3(nty), dim3(64 * push_waves(16)), 0, s, w, ntx, col);
        break;
    default:
        hipLaunchKernelGGL((k_window_remove<32>), dim3(nty), dim3(64 * push_waves(32)), 0, s, w, ntx, col);
        break;
    }
}

void launch_place_new(const int32_t *src, int32_t *dst, int16_t *ldst, int n, int nx, int ny, int col, int tile,
                      int *err, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(k_place_new, dim3((n + 255) / 256), dim3(256), 0, s, src, dst, ldst, n, nx, ny, col, tile,
                           err);
}

}  // namespace pic

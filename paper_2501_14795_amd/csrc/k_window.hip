// The moving-window step at the end of Listing 3.1: the window advances one
// cell towards +x, so the fields and the particles move one cell towards -x
// in window coordinates.  The particles that were in column 0 leave; the new
// particles (supplied by the caller) come in at column nx - 1.  The particle
// half produces exactly what the push kernel produces for the sort --
// per-wavefront leaver sub-lists in slot order, leaver copies and count
// records -- so the same canonical sort re-groups the particles by tile.
// Rare (once per cell of travel), so plain code: no LDS buffering.
#include "pic_internal.h"

namespace pic {

// tmp[c][j][i] = fld[c][j][i + 1] for the six E and B planes, zero at i = nx - 1
__global__ void __launch_bounds__(256) k_shift_fields(const float *__restrict__ fld, float *__restrict__ tmp, int nx,
                                                      int ny)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= nx || j >= ny) return;
    const int64_t P = (int64_t)nx * ny;
    const int64_t k = (int64_t)j * nx + i;
    for (int c = 0; c < 6; ++c) tmp[c * P + k] = i + 1 < nx ? fld[c * P + k + 1] : 0.0f;
}

// One tile per workgroup of push_waves(T) wavefronts, each streaming the run
// of the section the push kernel would give it (same leaver sub-list layout).
// Direction of a particle: 4 (stays: the cell to its left is in the same
// tile), 3 (the tile to the left), kDirRemoved (it was in column 0).
template <int T>
__global__ void __launch_bounds__(64 * push_waves(T)) k_window_shift(WindowSpecies w, int ntx, int *err)
{
    constexpr int W = push_waves(T);
    __shared__ int s_wl[W];
    __shared__ int s_left, s_removed;
    const int tile = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (threadIdx.x == 0) {
        s_left = 0;
        s_removed = 0;
    }
    __syncthreads();
    const int begin = w.off[tile], end = w.off[tile + 1];
    const int gx0 = (tile % ntx) * T;
    int lo, hi;
    wave_range(begin, end, wave, W, lo, hi);
    int nleav = 0, nleft = 0, nrem = 0;   // wavefront-uniform
    for (int cb = (lo >> 6) << 6; cb < hi; cb += 64) {
        const int i = cb + lane;
        const bool act = i >= lo && i < hi;
        int d = 4, nc = 0;
        if (act) {
            const int cell = w.p.cell[i];
            const int ix = cell & 0xffff, iy = cell >> 16;
            if (cell < 0 || ix - gx0 < 0 || ix - gx0 >= T) atomicOr(err, kErrOrder);
            d = ix == 0 ? kDirRemoved : (ix == gx0 ? 3 : 4);
            nc = d == kDirRemoved ? -1 : ((ix - 1) | (iy << 16));
            w.p.cell[i] = nc;
        }
        const bool leaves = act && d != 4;
        const unsigned long long m = __ballot(leaves);
        if (leaves) {
            const int64_t q = (int64_t)lo + nleav + (int)__builtin_amdgcn_mbcnt_hi(
                                  (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            w.leav[q] = ((uint32_t)(i - begin) << 4) | (uint32_t)d;
            w.lp.cell[q] = nc;
            w.lp.x[q] = w.p.x[i];
            w.lp.y[q] = w.p.y[i];
            w.lp.ux[q] = w.p.ux[i];
            w.lp.uy[q] = w.p.uy[i];
            w.lp.uz[q] = w.p.uz[i];
        }
        nleav += __popcll(m);
        nleft += __popcll(__ballot(act && d == 3));
        nrem += __popcll(__ballot(act && d == kDirRemoved));
    }
    if (lane == 0) {
        s_wl[wave] = nleav;
        atomicAdd(&s_left, nleft);
        atomicAdd(&s_removed, nrem);
    }
    __syncthreads();
    if (threadIdx.x < kCntStride) {
        const int k = threadIdx.x;
        int leavers = 0;
        for (int q = 0; q < W; ++q) leavers += s_wl[q];
        int v = 0;
        if (k < 9) v = k == 4 ? (end - begin) - leavers : (k == 3 ? s_left : 0);
        else if (k == kCntLeavers) v = leavers;
        else if (k >= kCntSub && k < kCntSub + W) v = s_wl[k - kCntSub];
        w.cnt[(int64_t)tile * kCntStride + k] = v;
    }
    if (threadIdx.x == 0 && s_removed) atomicAdd(w.removed, s_removed);
}

// every new particle must sit in column nx - 1
__global__ void __launch_bounds__(256) k_check_column(const int32_t *__restrict__ cell, int n, int nx, int *err)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && (cell[i] & 0xffff) != nx - 1) atomicOr(err, kErrOrder);
}

void launch_shift_fields(const float *fld, float *tmp, int nx, int ny, hipStream_t s)
{
    hipLaunchKernelGGL(k_shift_fields, dim3((nx + 63) / 64, (ny + 3) / 4), dim3(256), 0, s, fld, tmp, nx, ny);
}

void launch_window_shift(int tile, const WindowSpecies &w, int nx, int ntx, int n_tiles, int *err, hipStream_t s)
{
    (void)nx;
    if (n_tiles <= 0) return;
    switch (tile) {
    case 8: hipLaunchKernelGGL((k_window_shift<8>), dim3(n_tiles), dim3(64 * push_waves(8)), 0, s, w, ntx, err); break;
    case 16:
        hipLaunchKernelGGL((k_window_shift<16>), dim3(n_tiles), dim3(64 * push_waves(16)), 0, s, w, ntx, err);
        break;
    default:
        hipLaunchKernelGGL((k_window_shift<32>), dim3(n_tiles), dim3(64 * push_waves(32)), 0, s, w, ntx, err);
        break;
    }
}

void launch_check_column(const int32_t *cell, int n, int nx, int *err, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_check_column, dim3((n + 255) / 256), dim3(256), 0, s, cell, n, nx, err);
}

}  // namespace pic

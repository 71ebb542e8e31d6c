// The periodic fold of the tile current halos (update_gc_add of Listing
// 3.1), per node: shared by the J fold kernel (k_push.hip) and the fused
// field advance (k_field.hip), so both give J bit for bit alike.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

// J at node (gx, gy) = the sum over the tiles whose current halo (relative
// nodes -H..T+H, (T+2H+1)^2 per component, tile by tile in jtile) covers the
// node, in fixed (ty, tx) order with compensation.  A node at tile-relative
// (rx, ry) is covered by its own tile and, along x, by the left neighbour
// when rx <= H or the right one when rx >= T-H (never both: 2H + 1 <= T),
// likewise along y: at most 2 x 2 halos, whose values are all loaded before
// the sums (absent ones as zero, which leaves a compensated sum unchanged).
template <int T, int H>
__device__ __forceinline__ void fold_node(const float *__restrict__ jtile, int nx, int ny, int ntx, int nty, int gx,
                                          int gy, float out[3])
{
    (void)nx;
    (void)ny;
    constexpr int NJ = T + 2 * H + 1;
    constexpr int JP = NJ * NJ;
    const int bx = gx / T, by = gy / T;
    const int rx = gx - bx * T, ry = gy - by * T;
    // the two candidate offsets per axis, ascending: (-1, 0), (0, +1) or (0, none)
    const int kx0 = rx <= H ? -1 : 0, kx1 = rx <= H ? 0 : (rx >= T - H ? 1 : 0);
    const bool hx = rx <= H || rx >= T - H;
    const int ky0 = ry <= H ? -1 : 0, ky1 = ry <= H ? 0 : (ry >= T - H ? 1 : 0);
    const bool hy = ry <= H || ry >= T - H;
    float v[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int ky = (q >> 1) ? ky1 : ky0, kx = (q & 1) ? kx1 : kx0;
        const bool valid = ((q >> 1) == 0 || hy) && ((q & 1) == 0 || hx);
        int ty = by + ky, tx = bx + kx;
        ty = ty < 0 ? ty + nty : (ty >= nty ? ty - nty : ty);
        tx = tx < 0 ? tx + ntx : (tx >= ntx ? tx - ntx : tx);
        const int ly = ry - ky * T, lx = rx - kx * T;   // in -H..T+H
        const float *src = jtile + (int64_t)(ty * ntx + tx) * 3 * JP + (ly + H) * NJ + (lx + H);
#pragma unroll
        for (int c = 0; c < 3; ++c) v[q][c] = valid ? src[c * JP] : 0.0f;
    }
    float sum[3] = {0.0f, 0.0f, 0.0f}, cmp[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float x = v[q][c];
            const float t = sum[c] + x;
            const float bp = t - sum[c];
            cmp[c] += (sum[c] - (t - bp)) + (x - bp);
            sum[c] = t;
        }
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c] = sum[c] + cmp[c];
}

}  // namespace pic

// Yee field update on the periodic staggered grid (Eqs. 19-20; the three
// sub-steps of Listing 3.1 are three launches).  One thread per cell, the
// periodic neighbours read directly (this replaces the guard-cell copy).
// Outside the particle hot path: a plain coalesced stencil.
#include "pic_internal.h"

namespace pic {

// Faraday: B -= h curl E for one 64 x 4 block of cells (hdx = h/dx, hdy = h/dy).
__device__ __forceinline__ void yee_b_block(const FieldArgs &a, int bx, int by)
{
    const int i = bx * 64 + (threadIdx.x & 63);
    const int j = by * 4 + (threadIdx.x >> 6);
    const int nx = a.nx, ny = a.ny;
    if (i >= nx || j >= ny) return;
    float *__restrict__ f = a.fld;
    const int64_t P = (int64_t)nx * ny;
    const int64_t k = (int64_t)j * nx + i;
    const int64_t kx = (int64_t)j * nx + (i + 1 == nx ? 0 : i + 1);
    const int64_t ky = (int64_t)(j + 1 == ny ? 0 : j + 1) * nx + i;
    const float *Ex = f, *Ey = f + P, *Ez = f + 2 * P;
    float *Bx = f + 3 * P, *By = f + 4 * P, *Bz = f + 5 * P;
    const float ez = Ez[k];
    Bx[k] -= a.hdy * (Ez[ky] - ez);
    By[k] += a.hdx * (Ez[kx] - ez);
    Bz[k] -= a.hdx * (Ey[kx] - Ey[k]) - a.hdy * (Ex[ky] - Ex[k]);
}

// Ampere: E += dt (curl B - J) for one 64 x 4 block of cells.
__device__ __forceinline__ void yee_e_block(const FieldArgs &a, int bx, int by)
{
    const int i = bx * 64 + (threadIdx.x & 63);
    const int j = by * 4 + (threadIdx.x >> 6);
    const int nx = a.nx, ny = a.ny;
    if (i >= nx || j >= ny) return;
    float *__restrict__ f = a.fld;
    const int64_t P = (int64_t)nx * ny;
    const int64_t k = (int64_t)j * nx + i;
    const int64_t kx = (int64_t)j * nx + (i == 0 ? nx - 1 : i - 1);
    const int64_t ky = (int64_t)(j == 0 ? ny - 1 : j - 1) * nx + i;
    float *Ex = f, *Ey = f + P, *Ez = f + 2 * P;
    const float *Bx = f + 3 * P, *By = f + 4 * P, *Bz = f + 5 * P;
    const float *Jx = f + 6 * P, *Jy = f + 7 * P, *Jz = f + 8 * P;
    const float bz = Bz[k];
    Ex[k] += a.dtdy * (bz - Bz[ky]) - a.dt * Jx[k];
    Ey[k] += -a.dtdx * (bz - Bz[kx]) - a.dt * Jy[k];
    Ez[k] += a.dtdx * (By[k] - By[kx]) - a.dtdy * (Bx[k] - Bx[ky]) - a.dt * Jz[k];
}

__global__ void __launch_bounds__(256) k_yee_b(FieldArgs a) { yee_b_block(a, blockIdx.x, blockIdx.y); }
__global__ void __launch_bounds__(256) k_yee_e(FieldArgs a) { yee_e_block(a, blockIdx.x, blockIdx.y); }

// many simulations: items = (simulation, bx, by)
__global__ void __launch_bounds__(256) k_yee_b_b(const FieldArgs *d, const int4 *it)
{
    const int4 w = it[blockIdx.x];
    yee_b_block(d[w.x], w.y, w.z);
}
__global__ void __launch_bounds__(256) k_yee_e_b(const FieldArgs *d, const int4 *it)
{
    const int4 w = it[blockIdx.x];
    yee_e_block(d[w.x], w.y, w.z);
}

void launch_field_advance(const FieldArgs &f, hipStream_t s)
{
    const dim3 grid((f.nx + 63) / 64, (f.ny + 3) / 4);
    hipLaunchKernelGGL(k_yee_b, grid, dim3(256), 0, s, f);
    hipLaunchKernelGGL(k_yee_e, grid, dim3(256), 0, s, f);
    hipLaunchKernelGGL(k_yee_b, grid, dim3(256), 0, s, f);
}

void launch_field_advance_batch(const FieldArgs *descs, const int4 *items, int n_items, hipStream_t s)
{
    if (n_items == 0) return;
    hipLaunchKernelGGL(k_yee_b_b, dim3(n_items), dim3(256), 0, s, descs, items);
    hipLaunchKernelGGL(k_yee_e_b, dim3(n_items), dim3(256), 0, s, descs, items);
    hipLaunchKernelGGL(k_yee_b_b, dim3(n_items), dim3(256), 0, s, descs, items);
}

}  // namespace pic

// Yee field update on the periodic staggered grid (Eqs. 19-20; the three
// sub-steps of Listing 3.1 are three launches).  One thread per cell, the
// periodic neighbours read directly (this replaces the guard-cell copy).
// Outside the particle hot path: a plain coalesced stencil.
#include "pic_internal.h"

namespace pic {

// Faraday: B -= h curl E, with hdx = h/dx, hdy = h/dy.
__global__ void __launch_bounds__(256) k_yee_b(float *__restrict__ f, int nx, int ny, float hdx, float hdy)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= nx || j >= ny) return;
    const int64_t P = (int64_t)nx * ny;
    const int64_t k = (int64_t)j * nx + i;
    const int64_t kx = (int64_t)j * nx + (i + 1 == nx ? 0 : i + 1);
    const int64_t ky = (int64_t)(j + 1 == ny ? 0 : j + 1) * nx + i;
    const float *Ex = f, *Ey = f + P, *Ez = f + 2 * P;
    float *Bx = f + 3 * P, *By = f + 4 * P, *Bz = f + 5 * P;
    const float ez = Ez[k];
    Bx[k] -= hdy * (Ez[ky] - ez);
    By[k] += hdx * (Ez[kx] - ez);
    Bz[k] -= hdx * (Ey[kx] - Ey[k]) - hdy * (Ex[ky] - Ex[k]);
}

// Ampere: E += dt (curl B - J), with dtdx = dt/dx, dtdy = dt/dy.
__global__ void __launch_bounds__(256) k_yee_e(float *__restrict__ f, int nx, int ny, float dt, float dtdx,
                                               float dtdy)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= nx || j >= ny) return;
    const int64_t P = (int64_t)nx * ny;
    const int64_t k = (int64_t)j * nx + i;
    const int64_t kx = (int64_t)j * nx + (i == 0 ? nx - 1 : i - 1);
    const int64_t ky = (int64_t)(j == 0 ? ny - 1 : j - 1) * nx + i;
    float *Ex = f, *Ey = f + P, *Ez = f + 2 * P;
    const float *Bx = f + 3 * P, *By = f + 4 * P, *Bz = f + 5 * P;
    const float *Jx = f + 6 * P, *Jy = f + 7 * P, *Jz = f + 8 * P;
    const float bz = Bz[k];
    Ex[k] += dtdy * (bz - Bz[ky]) - dt * Jx[k];
    Ey[k] += -dtdx * (bz - Bz[kx]) - dt * Jy[k];
    Ez[k] += dtdx * (By[k] - By[kx]) - dtdy * (Bx[k] - Bx[ky]) - dt * Jz[k];
}

void launch_yee_b(float *fld, int nx, int ny, float hdx, float hdy, hipStream_t s)
{
    hipLaunchKernelGGL(k_yee_b, dim3((nx + 63) / 64, (ny + 3) / 4), dim3(256), 0, s, fld, nx, ny, hdx, hdy);
}

void launch_yee_e(float *fld, int nx, int ny, float dt, float dtdx, float dtdy, hipStream_t s)
{
    hipLaunchKernelGGL(k_yee_e, dim3((nx + 63) / 64, (ny + 3) / 4), dim3(256), 0, s, fld, nx, ny, dt, dtdx,
                       dtdy);
}

}  // namespace pic

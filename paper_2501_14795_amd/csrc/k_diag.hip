// Diagnostics with FP64 accumulation (energies, node charge density, the
// discrete continuity residual of Eq. 12, the residuals of Gauss's law and of
// div B = 0).  Not on the hot path.
#include "pic_internal.h"

namespace pic {

__device__ double block_sum_d(double v)
{
    __shared__ double s[16];
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_down(v, d, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) s[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += s[k];
    return t;
}

__device__ void atomic_max_nonneg(double *p, double v)
{
    // non-negative doubles order like their bit patterns
    atomicMax((unsigned long long *)p, (unsigned long long)__double_as_longlong(v));
}

__global__ void __launch_bounds__(256) k_field_energy(const float *__restrict__ f, int64_t plane, double *acc)
{
    double se = 0.0, sb = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < 3 * plane;
         k += (int64_t)gridDim.x * blockDim.x) {
        const double e = f[k], b = f[3 * plane + k];
        se += e * e;
        sb += b * b;
    }
    se = block_sum_d(se);
    __syncthreads();
    sb = block_sum_d(sb);
    if (threadIdx.x == 0) {
        atomicAdd(&acc[0], se);
        atomicAdd(&acc[1], sb);
    }
}

__global__ void __launch_bounds__(256) k_kinetic(DiagSpecies sp, double *acc)
{
    double s = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < sp.n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const double ux = sp.ux[p], uy = sp.uy[p], uz = sp.uz[p];
        const double u2 = ux * ux + uy * uy + uz * uz;
        s += u2 / (sqrt(1.0 + u2) + 1.0);   // gamma - 1 without cancellation
    }
    s = block_sum_d(s);
    if (threadIdx.x == 0) atomicAdd(acc, s);
}

__global__ void __launch_bounds__(256) k_rho(DiagSpecies sp, int nx, int ny, double *rho)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= sp.n) return;
    const int c = sp.cell[p];
    const int i0 = c & 0xffff, j0 = c >> 16;
    if ((unsigned)i0 >= (unsigned)nx || (unsigned)j0 >= (unsigned)ny) return;
    const double x = sp.x[p], y = sp.y[p], q = sp.q;
    if (sp.quadratic) {
        // the three nodes nearest the particle on each axis, weighted by the
        // quadratic B-spline at their distance
        const int hx = x >= 0.5 ? 1 : 0, hy = y >= 0.5 ? 1 : 0;
        const double ex = x - hx, ey = y - hy;   // offset from the nearest node, [-1/2, 1/2)
        const double wx[3] = {0.5 * (0.5 - ex) * (0.5 - ex), 0.75 - ex * ex, 0.5 * (0.5 + ex) * (0.5 + ex)};
        const double wy[3] = {0.5 * (0.5 - ey) * (0.5 - ey), 0.75 - ey * ey, 0.5 * (0.5 + ey) * (0.5 + ey)};
        for (int b = 0; b < 3; ++b) {
            int j = j0 + hy + b - 1;
            j = j < 0 ? j + ny : (j >= ny ? j - ny : j);
            for (int a = 0; a < 3; ++a) {
                int i = i0 + hx + a - 1;
                i = i < 0 ? i + nx : (i >= nx ? i - nx : i);
                atomicAdd(&rho[(int64_t)j * nx + i], q * wx[a] * wy[b]);
            }
        }
        return;
    }
    const int i1 = i0 + 1 == nx ? 0 : i0 + 1, j1 = j0 + 1 == ny ? 0 : j0 + 1;
    atomicAdd(&rho[(int64_t)j0 * nx + i0], q * (1.0 - x) * (1.0 - y));
    atomicAdd(&rho[(int64_t)j0 * nx + i1], q * x * (1.0 - y));
    atomicAdd(&rho[(int64_t)j1 * nx + i0], q * (1.0 - x) * y);
    atomicAdd(&rho[(int64_t)j1 * nx + i1], q * x * y);
}

__global__ void __launch_bounds__(256) k_continuity(const double *rho_prev, const double *rho_now,
                                                    const float *J, int nx, int ny, double dt, double dx,
                                                    double dy, double *acc)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= nx || j >= ny) return;
    const int64_t P = (int64_t)nx * ny;
    const int64_t k = (int64_t)j * nx + i;
    const int64_t kx = (int64_t)j * nx + (i == 0 ? nx - 1 : i - 1);
    const int64_t ky = (int64_t)(j == 0 ? ny - 1 : j - 1) * nx + i;
    const double div = ((double)J[k] - (double)J[kx]) / dx + ((double)J[P + k] - (double)J[P + ky]) / dy;
    const double r = rho_now[k] - rho_prev[k] + dt * div;
    atomic_max_nonneg(&acc[0], fabs(r));
    atomic_max_nonneg(&acc[1], fabs(rho_now[k]));
}

// Gauss's law residual at the nodes, div E - (rho - rho_bar) with the ions a
// uniform neutralising background rho_bar, and div B at the cell centres
// (i+1/2, j+1/2); maxima of their magnitudes into acc[0], acc[1].
__global__ void __launch_bounds__(256) k_gauss(const float *__restrict__ f, const double *rho, double rho_bar,
                                               int nx, int ny, double dx, double dy, double *acc)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= nx || j >= ny) return;
    const int64_t P = (int64_t)nx * ny;
    const int64_t k = (int64_t)j * nx + i;
    const int64_t kxm = (int64_t)j * nx + (i == 0 ? nx - 1 : i - 1);
    const int64_t kym = (int64_t)(j == 0 ? ny - 1 : j - 1) * nx + i;
    const int64_t kxp = (int64_t)j * nx + (i + 1 == nx ? 0 : i + 1);
    const int64_t kyp = (int64_t)(j + 1 == ny ? 0 : j + 1) * nx + i;
    const double dive = ((double)f[k] - (double)f[kxm]) / dx + ((double)f[P + k] - (double)f[P + kym]) / dy;
    const double divb = ((double)f[3 * P + kxp] - (double)f[3 * P + k]) / dx +
                        ((double)f[4 * P + kyp] - (double)f[4 * P + k]) / dy;
    atomic_max_nonneg(&acc[0], fabs(dive - (rho[k] - rho_bar)));
    atomic_max_nonneg(&acc[1], fabs(divb));
}

__global__ void __launch_bounds__(256) k_counts(const int32_t *cnt, const int32_t *mcount, int n_tiles,
                                                unsigned long long *acc)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    atomicAdd(&acc[0], (unsigned long long)cnt[(int64_t)t * kCntStride + kCntLeavers]);
    atomicAdd(&acc[1], (unsigned long long)mcount[t]);
}

static int grid_for(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 4096); }

void launch_diag_field_energy(const float *fld, int64_t plane, double *acc, hipStream_t s)
{
    hipLaunchKernelGGL(k_field_energy, dim3(grid_for(3 * plane)), dim3(256), 0, s, fld, plane, acc);
}

void launch_diag_kinetic(const DiagSpecies &sp, double *acc, hipStream_t s)
{
    if (sp.n > 0) hipLaunchKernelGGL(k_kinetic, dim3(grid_for(sp.n)), dim3(256), 0, s, sp, acc);
}

void launch_diag_rho(const DiagSpecies &sp, int nx, int ny, double *rho, hipStream_t s)
{
    if (sp.n > 0) hipLaunchKernelGGL(k_rho, dim3((sp.n + 255) / 256), dim3(256), 0, s, sp, nx, ny, rho);
}

void launch_diag_continuity(const double *rho_prev, const double *rho_now, const float *J, int nx, int ny,
                            double dt, double dx, double dy, double *acc, hipStream_t s)
{
    hipLaunchKernelGGL(k_continuity, dim3((nx + 63) / 64, (ny + 3) / 4), dim3(256), 0, s, rho_prev, rho_now,
                       J, nx, ny, dt, dx, dy, acc);
}

void launch_diag_gauss(const float *fld, const double *rho, double rho_bar, int nx, int ny, double dx, double dy,
                       double *acc, hipStream_t s)
{
    hipLaunchKernelGGL(k_gauss, dim3((nx + 63) / 64, (ny + 3) / 4), dim3(256), 0, s, fld, rho, rho_bar, nx, ny,
                       dx, dy, acc);
}

void launch_diag_counts(const int32_t *cnt, const int32_t *mcount, int n_tiles, unsigned long long *acc,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_counts, dim3((n_tiles + 255) / 256), dim3(256), 0, s, cnt, mcount, n_tiles, acc);
}

}  // namespace pic

// Valid initial fields (Sec. 3.2: before the first step the fields satisfy
// Eq. 17, div E = rho, and Eq. 18, div B = 0).  Both are projections onto
// the periodic grid's gradients: E <- E - grad psi with Lap psi = div E -
// (rho - <rho>) (psi at the nodes) and B <- B - grad chi with Lap chi = div B
// (chi at the cell centres), Lap the five-point Laplacian -- the divergence of
// the Yee gradient.  A gradient has no discrete curl, so the curls that drive
// Eqs. 19-20 are kept.
//
// The Poisson problems are solved by conjugate gradients in FP64.  Every
// scalar stays on the device: each dot product is a per-block partial sum
// followed by a one-block sum in fixed order (bit-reproducible), and the two
// r.r values of an iteration live in slots chosen by its parity, so no kernel
// overwrites a scalar another block may still read.  Support code for the
// initial state: plain grid-stride kernels.
#include "pic_internal.h"

namespace pic {

namespace {

constexpr int kCgBlock = 256;

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Sum of v over the block, written by thread 0 to out[blockIdx.x].
__device__ __forceinline__ void block_partial(double v, double *out)
{
    __shared__ double s[kCgBlock / 64];
    for (int d = 32; d > 0; d >>= 1) v += __shfl_down(v, d, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kCgBlock / 64; ++w) t += s[w];
        out[blockIdx.x] = t;
    }
}

// Right-hand sides.  E: r = div E - (rho - rho_bar) at the nodes, div E =
// (Ex[i] - Ex[i-1]) / dx + (Ey[j] - Ey[j-1]) / dy.  B: r = div B at the cell
// centres, (Bx[i+1] - Bx[i]) / dx + (By[j+1] - By[j]) / dy.  Partial sums of r.
__global__ void __launch_bounds__(kCgBlock) k_cg_rhs(const float *__restrict__ fld, const double *__restrict__ rho,
                                                     double rho_bar, int magnetic, int nx, int ny, double idx,
                                                     double idy, double *__restrict__ r, double *partial)
{
    const int64_t P = (int64_t)nx * ny;
    const float *fx = fld + (magnetic ? 3 * P : 0), *fy = fx + P;
    double acc = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P; k += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(k / nx), i = (int)(k - (int64_t)j * nx);
        double v;
        if (magnetic) {
            const int64_t kx = (int64_t)j * nx + wrap(i + 1, nx), ky = (int64_t)wrap(j + 1, ny) * nx + i;
            v = ((double)fx[kx] - (double)fx[k]) * idx + ((double)fy[ky] - (double)fy[k]) * idy;
        } else {
            const int64_t kx = (int64_t)j * nx + wrap(i - 1, nx), ky = (int64_t)wrap(j - 1, ny) * nx + i;
            v = ((double)fx[k] - (double)fx[kx]) * idx + ((double)fy[k] - (double)fy[ky]) * idy -
                (rho[k] - rho_bar);
        }
        r[k] = v;
        acc += v;
    }
    block_partial(acc, partial);
}

// The periodic Laplacian maps onto zero-mean grids only: remove the mean of r
// (round-off of the sums above), then x = 0, p = r; partial r.r.
__global__ void __launch_bounds__(kCgBlock) k_cg_center(double *__restrict__ x, double *__restrict__ r,
                                                        double *__restrict__ p, int64_t P,
                                                        const double *__restrict__ sum, double *partial)
{
    const double mean = *sum / (double)P;
    double acc = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P; k += (int64_t)gridDim.x * blockDim.x) {
        const double v = r[k] - mean;
        x[k] = 0.0;
        r[k] = v;
        p[k] = v;
        acc = fma(v, v, acc);
    }
    block_partial(acc, partial);
}

// One block: out = sum of the n partials, in index order.
__global__ void __launch_bounds__(kCgBlock) k_cg_sum(const double *__restrict__ partial, int n, double *out)
{
    double v = 0.0;
    for (int b = threadIdx.x; b < n; b += kCgBlock) v += partial[b];
    __shared__ double s[kCgBlock];
    s[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int b = 0; b < kCgBlock; ++b) t += s[b];
        *out = t;
    }
}

// q = Lap p (five-point, periodic), partial p.q
__global__ void __launch_bounds__(kCgBlock) k_cg_apply(const double *__restrict__ p, double *__restrict__ q, int nx,
                                                       int ny, double idx2, double idy2, double *partial)
{
    const int64_t P = (int64_t)nx * ny;
    double acc = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P; k += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(k / nx), i = (int)(k - (int64_t)j * nx);
        const int64_t row = (int64_t)j * nx;
        const double c = p[k];
        const double lx = p[row + wrap(i + 1, nx)] - 2.0 * c + p[row + wrap(i - 1, nx)];
        const double ly = p[(int64_t)wrap(j + 1, ny) * nx + i] - 2.0 * c + p[(int64_t)wrap(j - 1, ny) * nx + i];
        const double v = lx * idx2 + ly * idy2;
        q[k] = v;
        acc = fma(c, v, acc);
    }
    block_partial(acc, partial);
}

// alpha = rr / pq; x += alpha p; r -= alpha q; partial r.r
__global__ void __launch_bounds__(kCgBlock) k_cg_update(double *__restrict__ x, double *__restrict__ r,
                                                        const double *__restrict__ p, const double *__restrict__ q,
                                                        int64_t P, const double *__restrict__ scal, int cur,
                                                        double *partial)
{
    const double pq = scal[2], rr = scal[cur];
    const double alpha = pq != 0.0 ? rr / pq : 0.0;
    double acc = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P; k += (int64_t)gridDim.x * blockDim.x) {
        x[k] = fma(alpha, p[k], x[k]);
        const double v = fma(-alpha, q[k], r[k]);
        r[k] = v;
        acc = fma(v, v, acc);
    }
    block_partial(acc, partial);
}

// beta = rr_new / rr; p = r + beta p
__global__ void __launch_bounds__(kCgBlock) k_cg_direction(double *__restrict__ p, const double *__restrict__ r,
                                                           int64_t P, const double *__restrict__ scal, int cur)
{
    const double rr = scal[cur], rn = scal[cur ^ 1];
    const double beta = rr != 0.0 ? rn / rr : 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = fma(beta, p[k], r[k]);
}

// E: Ex -= (psi[i+1] - psi[i]) / dx, Ey -= (psi[j+1] - psi[j]) / dy.
// B: Bx -= (chi[i] - chi[i-1]) / dx, By -= (chi[j] - chi[j-1]) / dy.
// In FP64, stored as FP32.
__global__ void __launch_bounds__(kCgBlock) k_cg_project(float *__restrict__ fld, const double *__restrict__ s,
                                                         int magnetic, int nx, int ny, double idx, double idy)
{
    const int64_t P = (int64_t)nx * ny;
    float *fx = fld + (magnetic ? 3 * P : 0), *fy = fx + P;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P; k += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(k / nx), i = (int)(k - (int64_t)j * nx);
        double gx, gy;
        if (magnetic) {
            gx = (s[k] - s[(int64_t)j * nx + wrap(i - 1, nx)]) * idx;
            gy = (s[k] - s[(int64_t)wrap(j - 1, ny) * nx + i]) * idy;
        } else {
            gx = (s[(int64_t)j * nx + wrap(i + 1, nx)] - s[k]) * idx;
            gy = (s[(int64_t)wrap(j + 1, ny) * nx + i] - s[k]) * idy;
        }
        fx[k] = (float)((double)fx[k] - gx);
        fy[k] = (float)((double)fy[k] - gy);
    }
}

int cg_blocks(int64_t P)
{
    const int64_t b = (P + kCgBlock - 1) / kCgBlock;
    return (int)(b < kCgPartials ? (b > 0 ? b : 1) : kCgPartials);
}

}  // namespace

// One projection (magnetic = 0: E with rho; 1: B).  Returns the iterations
// run and the final ||r|| / ||r0|| (0 when r0 = 0), or -1 iterations on a
// HIP error; converged when the ratio is at most tol.
CgResult cg_project(float *fld, const double *rho, double rho_bar, int magnetic, int nx, int ny, double dx, double dy,
                    double tol, int max_iter, const CgScratch &w, hipStream_t s)
{
    CgResult res{0, 0.0, false};
    const int64_t P = (int64_t)nx * ny;
    const int nb = cg_blocks(P);
    const double idx = 1.0 / dx, idy = 1.0 / dy;
    hipLaunchKernelGGL(k_cg_rhs, dim3(nb), dim3(kCgBlock), 0, s, fld, rho, rho_bar, magnetic, nx, ny, idx, idy, w.r,
                       w.partial);
    hipLaunchKernelGGL(k_cg_sum, dim3(1), dim3(kCgBlock), 0, s, w.partial, nb, w.scal + 3);
    hipLaunchKernelGGL(k_cg_center, dim3(nb), dim3(kCgBlock), 0, s, w.x, w.r, w.p, P, w.scal + 3, w.partial);
    hipLaunchKernelGGL(k_cg_sum, dim3(1), dim3(kCgBlock), 0, s, w.partial, nb, w.scal + 0);
    double rr0 = 0.0;
    if (hipMemcpyAsync(&rr0, w.scal, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        res.iterations = -1;
        return res;
    }
    if (!(rr0 > 0.0)) {
        res.converged = true;
        return res;
    }
    const double goal = tol * tol * rr0;
    double rr = rr0;
    int k = 0;
    while (k < max_iter) {
        const int cur = k & 1;
        hipLaunchKernelGGL(k_cg_apply, dim3(nb), dim3(kCgBlock), 0, s, w.p, w.q, nx, ny, idx * idx, idy * idy,
                           w.partial);
        hipLaunchKernelGGL(k_cg_sum, dim3(1), dim3(kCgBlock), 0, s, w.partial, nb, w.scal + 2);
        hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(kCgBlock), 0, s, w.x, w.r, w.p, w.q, P, w.scal, cur,
                           w.partial);
        hipLaunchKernelGGL(k_cg_sum, dim3(1), dim3(kCgBlock), 0, s, w.partial, nb, w.scal + (cur ^ 1));
        hipLaunchKernelGGL(k_cg_direction, dim3(nb), dim3(kCgBlock), 0, s, w.p, w.r, P, w.scal, cur);
        ++k;
        if ((k & 15) == 0 || k == max_iter) {
            if (hipMemcpyAsync(&rr, w.scal + (k & 1), sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                res.iterations = -1;
                return res;
            }
            if (rr <= goal) break;
        }
    }
    res.iterations = k;
    res.residual = sqrt(rr / rr0);
    res.converged = rr <= goal;
    hipLaunchKernelGGL(k_cg_project, dim3(nb), dim3(kCgBlock), 0, s, fld, w.x, magnetic, nx, ny, idx, idy);
    return res;
}

}  // namespace pic

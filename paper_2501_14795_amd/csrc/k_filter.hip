// Binomial filter (Listing 3.1: the optional smoothing of J after
// update_gc_add).  One pass smooths each plane with the three-point kernel
// (1/4, 1/2, 1/4) along x and then along y on the periodic grid; here both
// directions are one 3 x 3 stencil evaluated in that order (row sums first),
// out of place, one launch per pass.  FP32 for the current; FP64 for the
// charge density of the diagnostics, which must be filtered alike for the
// continuity and Gauss residuals to hold.  A plain coalesced stencil, bound
// by HBM bandwidth.
#include "pic_internal.h"

namespace pic {

template <typename T>
__device__ __forceinline__ void binomial_block(const FilterArgs &a, int bx, int by)
{
    const int nx = a.nx, ny = a.ny;
    const int i = bx * 64 + (threadIdx.x & 63);
    const int j = by * 4 + (threadIdx.x >> 6);
    if (i >= nx || j >= ny) return;
    const int im = i == 0 ? nx - 1 : i - 1, ip = i + 1 == nx ? 0 : i + 1;
    const int64_t rm = (int64_t)(j == 0 ? ny - 1 : j - 1) * nx, r0 = (int64_t)j * nx,
                  rp = (int64_t)(j + 1 == ny ? 0 : j + 1) * nx;
    const int64_t P = (int64_t)nx * ny;
    const T q = (T)0.25, h = (T)0.5;
    for (int c = 0; c < a.planes; ++c) {
        const T *__restrict__ s = (const T *)a.src + c * P;
        const T sm = q * s[rm + im] + h * s[rm + i] + q * s[rm + ip];
        const T s0 = q * s[r0 + im] + h * s[r0 + i] + q * s[r0 + ip];
        const T sp = q * s[rp + im] + h * s[rp + i] + q * s[rp + ip];
        ((T *)a.dst)[c * P + r0 + i] = q * sm + h * s0 + q * sp;
    }
}

__global__ void __launch_bounds__(256) k_binomial_f(FilterArgs a) { binomial_block<float>(a, blockIdx.x, blockIdx.y); }
__global__ void __launch_bounds__(256) k_binomial_d(FilterArgs a) { binomial_block<double>(a, blockIdx.x, blockIdx.y); }

// many simulations (FP32 current): items = (simulation, bx, by) over 64 x 4 blocks
__global__ void __launch_bounds__(256) k_binomial_f_b(const FilterArgs *d, const int4 *it)
{
    const int4 w = it[blockIdx.x];
    binomial_block<float>(d[w.x], w.y, w.z);
}

void launch_filter(const FilterArgs &a, bool fp64, hipStream_t s)
{
    const dim3 grid((a.nx + 63) / 64, (a.ny + 3) / 4);
    if (fp64)
        hipLaunchKernelGGL(k_binomial_d, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_binomial_f, grid, dim3(256), 0, s, a);
}

void launch_filter_batch(const FilterArgs *descs, const int4 *items, int n_items, hipStream_t s)
{
    if (n_items > 0) hipLaunchKernelGGL(k_binomial_f_b, dim3(n_items), dim3(256), 0, s, descs, items);
}

}  // namespace pic

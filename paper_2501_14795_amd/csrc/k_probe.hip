// Streaming probe: the particle stream of the push kernel without the
// particle arithmetic -- one array of n 16-bit values (the tile-relative
// cells) and five of n 32-bit values, each read and written back in place,
// 64-element chunks per wavefront through raw buffer descriptors, with or
// without the non-temporal hint the push uses.  It measures the bandwidth
// that access pattern reaches on the device (the practical ceiling of the
// push's streaming), and leaves the data unchanged.
#include "pic_internal.h"

namespace pic {

namespace {

constexpr int kProbeBlock = 256;
constexpr int kProbeSlice = 1 << 14;
constexpr int kRsrcWord3Probe = 0x00020000;   // raw 32-bit buffer access, gfx9 family

template <int CPOL>
__global__ void __launch_bounds__(kProbeBlock) k_probe_stream(uint16_t *a0, float *a1, float *a2, float *a3,
                                                              float *a4, float *a5, int64_t n)
{
    // each block streams its own slice of kProbeSlice elements of every
    // array, as a workgroup of the push streams a 32 x 32 tile's section
    constexpr int64_t kSlice = kProbeSlice;
    const int64_t b0 = (int64_t)blockIdx.x * kSlice;
    if (b0 >= n) return;
    const int len = (int)min(kSlice, n - b0);
    float *base[6] = {nullptr, a1, a2, a3, a4, a5};
    __amdgpu_buffer_rsrc_t r[6];
    r[0] = __builtin_amdgcn_make_buffer_rsrc(a0 + b0, (short)0, len * 2, kRsrcWord3Probe);
#pragma unroll
    for (int k = 1; k < 6; ++k)
        r[k] = __builtin_amdgcn_make_buffer_rsrc(base[k] + b0, (short)0, len * 4, kRsrcWord3Probe);
    for (int i = threadIdx.x; i < len; i += 2 * kProbeBlock) {
        unsigned v[2][6];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int k = 0; k < 6; ++k)
                v[u][k] = k == 0 ? __builtin_amdgcn_raw_buffer_load_b16(r[0], (i + u * kProbeBlock) * 2, 0, CPOL)
                                 : __builtin_amdgcn_raw_buffer_load_b32(r[k], (i + u * kProbeBlock) * 4, 0, CPOL);
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int k = 0; k < 6; ++k)
                if (i + u * kProbeBlock < len) {
                    if (k == 0)
                        __builtin_amdgcn_raw_buffer_store_b16((unsigned short)v[u][0], r[0],
                                                              (i + u * kProbeBlock) * 2, 0, CPOL);
                    else
                        __builtin_amdgcn_raw_buffer_store_b32(v[u][k], r[k], (i + u * kProbeBlock) * 4, 0, CPOL);
                }
    }
}

}  // namespace

}  // namespace pic

extern "C" int pic_probe_stream(void *const *arrays, int64_t n, int nontemporal, hipStream_t stream)
{
    using namespace pic;
    if (!arrays || n < 0) return PIC_EINVAL;
    for (int k = 0; k < 6; ++k)
        if (!arrays[k] && n > 0) return PIC_EINVAL;
    if (n == 0) return PIC_OK;
    const int64_t blocks = (n + kProbeSlice - 1) / kProbeSlice;
    if (blocks > 0x7fffffff) return PIC_EINVAL;
    if (nontemporal)
        hipLaunchKernelGGL(k_probe_stream<2>, dim3((unsigned)blocks), dim3(kProbeBlock), 0, stream,
                           (uint16_t *)arrays[0], (float *)arrays[1], (float *)arrays[2], (float *)arrays[3],
                           (float *)arrays[4], (float *)arrays[5], n);
    else
        hipLaunchKernelGGL(k_probe_stream<0>, dim3((unsigned)blocks), dim3(kProbeBlock), 0, stream,
                           (uint16_t *)arrays[0], (float *)arrays[1], (float *)arrays[2], (float *)arrays[3],
                           (float *)arrays[4], (float *)arrays[5], n);
    return hipGetLastError() == hipSuccess ? PIC_OK : PIC_EHIP;
}

// Grouping caller particles by tile (Sec. 4.1: the particles of a tile
// occupy one contiguous section, sections in tile order, Fig. 4.3) when they
// arrive in any order: a stable least-significant-digit radix sort on the
// tile id, 8 bits per pass, then a gather of the six particle arrays.
// Stability keeps the given order inside a tile, so already grouped input is
// left as it is.  Runs at initialisation and state loads.
//
// One pass over n keys, in chunks of kTsChunk consecutive keys per
// workgroup:
//   hist    per chunk and digit, the number of keys -> hist[digit][chunk]
//   scan    exclusive prefix over hist in (digit, chunk) order: where each
//           chunk's keys of each digit start in the output
//   scatter each chunk walks its keys in index order, 1024 at a time: within
//           a wavefront the lanes holding the same digit are found with eight
//           ballots (one per digit bit) and ranked by lane; per-wavefront
//           digit counts in LDS rank the wavefronts; a running base per digit
//           carries over to the next 1024
#include "pic_internal.h"

namespace pic {

namespace {

constexpr int kTsThreads = 1024;                 // 16 wavefronts
constexpr int kTsRounds = 16;                    // keys per thread per chunk
constexpr int kTsChunk = kTsThreads * kTsRounds;
constexpr int kTsWaves = kTsThreads / 64;

__global__ void __launch_bounds__(256) k_ts_keys(const int32_t *__restrict__ cell, int n, int tsh, int ntx,
                                                 uint32_t *__restrict__ key, uint32_t *__restrict__ val)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = cell[i];
    key[i] = (uint32_t)(((c >> 16) >> tsh) * ntx + ((c & 0xffff) >> tsh));
    val[i] = (uint32_t)i;
}

__global__ void __launch_bounds__(kTsThreads) k_ts_hist(const uint32_t *__restrict__ key, int n, int shift,
                                                        int n_chunks, int32_t *__restrict__ hist)
{
    __shared__ int cnt[256];
    if (threadIdx.x < 256) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTsChunk;
    for (int r = 0; r < kTsRounds; ++r) {
        const int64_t i = base + (int64_t)r * kTsThreads + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(key[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    if (threadIdx.x < 256) hist[(int64_t)threadIdx.x * n_chunks + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan of 1024 values per block in place; block totals to bs.
__global__ void __launch_bounds__(1024) k_ts_scan_blocks(int32_t *__restrict__ v, int64_t len, int32_t *bs)
{
    __shared__ int s[kTsWaves];
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    const int x = i < len ? v[i] : 0;
    int incl = x;
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(incl, d, 64);
        if ((threadIdx.x & 63) >= d) incl += y;
    }
    if ((threadIdx.x & 63) == 63) s[threadIdx.x >> 6] = incl;
    __syncthreads();
    int wb = 0;
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) wb += s[w];
    if (i < len) v[i] = wb + incl - x;
    if (threadIdx.x == 1023) bs[blockIdx.x] = wb + incl;
}

// One block: exclusive scan of the nb block totals in place.
__global__ void __launch_bounds__(1024) k_ts_scan_top(int32_t *__restrict__ bs, int nb)
{
    __shared__ int s[kTsWaves];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int b0 = 0; b0 < nb; b0 += 1024) {
        const int b = b0 + threadIdx.x;
        const int x = b < nb ? bs[b] : 0;
        int incl = x;
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(incl, d, 64);
            if ((threadIdx.x & 63) >= d) incl += y;
        }
        if ((threadIdx.x & 63) == 63) s[threadIdx.x >> 6] = incl;
        __syncthreads();
        int wb = 0, tot = 0;
        for (int w = 0; w < kTsWaves; ++w) {
            if (w < (int)(threadIdx.x >> 6)) wb += s[w];
            tot += s[w];
        }
        const int c = carry;
        if (b < nb) bs[b] = c + wb + incl - x;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(1024) k_ts_scan_add(int32_t *__restrict__ v, int64_t len, const int32_t *bs)
{
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    if (i < len) v[i] += bs[blockIdx.x];
}

__global__ void __launch_bounds__(kTsThreads) k_ts_scatter(const uint32_t *__restrict__ key_in,
                                                           const uint32_t *__restrict__ val_in, int n, int shift,
                                                           int n_chunks, const int32_t *__restrict__ hist,
                                                           uint32_t *__restrict__ key_out,
                                                           uint32_t *__restrict__ val_out)
{
    __shared__ int base[256];
    __shared__ int wcnt[kTsWaves][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x < 256) base[threadIdx.x] = hist[(int64_t)threadIdx.x * n_chunks + blockIdx.x];
    const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int64_t cbase = (int64_t)blockIdx.x * kTsChunk;
    for (int r = 0; r < kTsRounds; ++r) {
        for (int e = threadIdx.x; e < kTsWaves * 256; e += kTsThreads) (&wcnt[0][0])[e] = 0;
        __syncthreads();
        const int64_t i = cbase + (int64_t)r * kTsThreads + threadIdx.x;
        const bool act = i < n;
        uint32_t k = 0, v = 0;
        int d = 0;
        if (act) {
            k = key_in[i];
            v = val_in[i];
            d = (int)((k >> shift) & 255u);
        }
        // lanes of this wavefront holding the same digit
        unsigned long long same = __ballot(act);
        for (int b = 0; b < 8; ++b) {
            const unsigned long long m = __ballot(act && ((d >> b) & 1));
            same &= ((d >> b) & 1) ? m : ~m;
        }
        const int rank = __popcll(same & below);
        if (act && rank == 0) wcnt[wave][d] = __popcll(same);
        __syncthreads();
        if (act) {
            int pos = base[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
            key_out[pos] = k;
            val_out[pos] = v;
        }
        __syncthreads();
        if (threadIdx.x < 256) {
            int t = 0;
            for (int w = 0; w < kTsWaves; ++w) t += wcnt[w][threadIdx.x];
            base[threadIdx.x] += t;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_ts_gather(GParts dst, GParts src, const uint32_t *__restrict__ perm, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t j = perm[i];
    dst.cell[i] = src.cell[j];
    dst.x[i] = src.x[j];
    dst.y[i] = src.y[j];
    dst.ux[i] = src.ux[j];
    dst.uy[i] = src.uy[j];
    dst.uz[i] = src.uz[j];
}

}  // namespace

int64_t tile_sort_hist_entries(int n)
{
    const int64_t chunks = ((int64_t)n + kTsChunk - 1) / kTsChunk;
    const int64_t len = 256 * chunks;
    return len + (len + 1023) / 1024;
}

const uint32_t *launch_tile_sort_perm(const TileSortArgs &a, hipStream_t s)
{
    const int n = a.n;
    if (n <= 1 || a.n_tiles <= 1) return nullptr;
    const int tsh = __builtin_ctz(a.tile);
    int bits = 0;
    while ((1 << bits) < a.n_tiles) ++bits;
    const int n_chunks = (int)(((int64_t)n + kTsChunk - 1) / kTsChunk);
    const int64_t len = 256 * (int64_t)n_chunks;
    const int nb = (int)((len + 1023) / 1024);
    int32_t *bs = a.hist + len;
    uint32_t *kin = a.key[0], *vin = a.val[0], *kout = a.key[1], *vout = a.val[1];
    hipLaunchKernelGGL(k_ts_keys, dim3((n + 255) / 256), dim3(256), 0, s, a.p.cell, n, tsh, a.ntx, kin, vin);
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_ts_hist, dim3(n_chunks), dim3(kTsThreads), 0, s, kin, n, shift, n_chunks, a.hist);
        hipLaunchKernelGGL(k_ts_scan_blocks, dim3(nb), dim3(1024), 0, s, a.hist, len, bs);
        hipLaunchKernelGGL(k_ts_scan_top, dim3(1), dim3(1024), 0, s, bs, nb);
        hipLaunchKernelGGL(k_ts_scan_add, dim3(nb), dim3(1024), 0, s, a.hist, len, bs);
        hipLaunchKernelGGL(k_ts_scatter, dim3(n_chunks), dim3(kTsThreads), 0, s, kin, vin, n, shift, n_chunks,
                           a.hist, kout, vout);
        uint32_t *t = kin;
        kin = kout;
        kout = t;
        t = vin;
        vin = vout;
        vout = t;
    }
    return vin;
}

void launch_tile_sort_gather(const TileSortArgs &a, const uint32_t *perm, hipStream_t s)
{
    const int n = a.n;
    if (!perm || n <= 1) return;
    // copy the particles aside and gather them back in the new order
    const size_t bytes = (size_t)n * 4;
    (void)hipMemcpyAsync(a.tmp.cell, a.p.cell, bytes, hipMemcpyDeviceToDevice, s);
    (void)hipMemcpyAsync(a.tmp.x, a.p.x, bytes, hipMemcpyDeviceToDevice, s);
    (void)hipMemcpyAsync(a.tmp.y, a.p.y, bytes, hipMemcpyDeviceToDevice, s);
    (void)hipMemcpyAsync(a.tmp.ux, a.p.ux, bytes, hipMemcpyDeviceToDevice, s);
    (void)hipMemcpyAsync(a.tmp.uy, a.p.uy, bytes, hipMemcpyDeviceToDevice, s);
    (void)hipMemcpyAsync(a.tmp.uz, a.p.uz, bytes, hipMemcpyDeviceToDevice, s);
    hipLaunchKernelGGL(k_ts_gather, dim3((n + 255) / 256), dim3(256), 0, s, a.p, a.tmp, perm, n);
}

void launch_tile_sort(const TileSortArgs &a, hipStream_t s)
{
    launch_tile_sort_gather(a, launch_tile_sort_perm(a, s), s);
}

}  // namespace pic

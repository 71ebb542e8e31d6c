// Yee field update on the periodic staggered grid (Eqs. 19-20; the three
// sub-steps of Listing 3.1 are three launches).  One thread per cell, the
// periodic neighbours read directly (this replaces the guard-cell copy).
// Outside the particle hot path: a plain coalesced stencil.  In a step
// without the current filter the E step also folds the tile current halos
// into J (update_gc_add, the same per-node sum as the fold kernel), so J is
// written once and not read back.
#include "pic_internal.h"
#include "pic_fold.h"
#include "pic_yee.h"

namespace pic {

// Faraday: B -= h curl E for one 64 x 4 block of cells (hdx = h/dx, hdy = h/dy),
// from the B planes in place, or from the push's half-step planes (a.bh) into
// the B planes.
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
    const float *Bin = a.bh ? a.bh : f + 3 * P;
    float *Bx = f + 3 * P, *By = f + 4 * P, *Bz = f + 5 * P;
    const BCell b = faraday_half(Bin[k], Bin[P + k], Bin[2 * P + k], Ex[k], Ex[ky], Ey[k], Ey[kx], Ez[k], Ez[kx],
                                 Ez[ky], a.hdx, a.hdy);
    Bx[k] = b.x;
    By[k] = b.y;
    Bz[k] = b.z;
}

// Ampere: E += dt (curl B - J) for one 64 x 4 block of cells.  FOLD: J is
// first folded from the tile current halos (tile edge T, halo pad H) and
// written to the J planes; else read from them.
template <bool FOLD, int T, int H>
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
    const float *Bh = a.bh ? a.bh : f + 3 * P;   // B at the half step
    const float *Bx = Bh, *By = Bh + P, *Bz = Bh + 2 * P;
    float *Jx = f + 6 * P, *Jy = f + 7 * P, *Jz = f + 8 * P;
    float jx, jy, jz;
    if constexpr (FOLD) {
        float jv[3];
        fold_node<T, H>(a.jtile, nx, ny, a.ntx, a.nty, i, j, jv);
        jx = jv[0];
        jy = jv[1];
        jz = jv[2];
        Jx[k] = jx;
        Jy[k] = jy;
        Jz[k] = jz;
    } else {
        jx = Jx[k];
        jy = Jy[k];
        jz = Jz[k];
    }
    const float bz = Bz[k];
    Ex[k] += a.dtdy * (bz - Bz[ky]) - a.dt * jx;
    Ey[k] += -a.dtdx * (bz - Bz[kx]) - a.dt * jy;
    Ez[k] += a.dtdx * (By[k] - By[kx]) - a.dtdy * (Bx[k] - Bx[ky]) - a.dt * jz;
}

__global__ void __launch_bounds__(256) k_yee_b(FieldArgs a) { yee_b_block(a, blockIdx.x, blockIdx.y); }

template <bool FOLD, int T, int H>
__global__ void __launch_bounds__(256) k_yee_e(FieldArgs a)
{
    yee_e_block<FOLD, T, H>(a, blockIdx.x, blockIdx.y);
}

// many simulations: items = (simulation, bx, by)
__global__ void __launch_bounds__(256) k_yee_b_b(const FieldArgs *d, const int4 *it)
{
    const int4 w = it[blockIdx.x];
    yee_b_block(d[w.x], w.y, w.z);
}

template <bool FOLD, int T, int H>
__global__ void __launch_bounds__(256) k_yee_e_b(const FieldArgs *d, const int4 *it)
{
    const int4 w = it[blockIdx.x];
    yee_e_block<FOLD, T, H>(d[w.x], w.y, w.z);
}

namespace {

// The sub-steps, single (one 64 x 4 block per cell block) or batched
// (items), with the E step of fold / tile T / halo pad H: the first B half
// step, the E step and the second B half step, or, when the push has formed
// the first half step (bh), the E step and the second half step only.
struct FieldLaunch {
    const FieldArgs *single;
    const FieldArgs *descs;
    const int4 *items;
    int n_items;
    bool bh;
    hipStream_t s;
    template <bool FOLD, int T, int H>
    void go() const
    {
        if constexpr (cadence_ok(T, H)) {
            if (single) {
                const dim3 grid((single->nx + 63) / 64, (single->ny + 3) / 4);
                if (!bh) hipLaunchKernelGGL(k_yee_b, grid, dim3(256), 0, s, *single);
                hipLaunchKernelGGL((k_yee_e<FOLD, T, H>), grid, dim3(256), 0, s, *single);
                hipLaunchKernelGGL(k_yee_b, grid, dim3(256), 0, s, *single);
            } else if (n_items > 0) {
                if (!bh) hipLaunchKernelGGL(k_yee_b_b, dim3(n_items), dim3(256), 0, s, descs, items);
                hipLaunchKernelGGL((k_yee_e_b<FOLD, T, H>), dim3(n_items), dim3(256), 0, s, descs, items);
                hipLaunchKernelGGL(k_yee_b_b, dim3(n_items), dim3(256), 0, s, descs, items);
            }
        }
    }
};

template <int T>
void field_h(const FieldLaunch &L, int halo)
{
    if (halo == 2) L.go<true, T, 2>();
    else if (halo == 4) L.go<true, T, 4>();
    else L.go<true, T, 1>();
}

void field_dispatch(const FieldLaunch &L, bool fold, int tile, int halo)
{
    if (!fold) {
        L.go<false, 8, 1>();
        return;
    }
    switch (tile) {
    case 8: field_h<8>(L, halo); break;
    case 16: field_h<16>(L, halo); break;
    default: field_h<32>(L, halo); break;
    }
}

}  // namespace

void launch_field_advance(const FieldArgs &f, int tile, int halo, hipStream_t s)
{
    FieldLaunch L{&f, nullptr, nullptr, 0, f.bh != nullptr, s};
    field_dispatch(L, f.jtile != nullptr, tile, halo);
}

void launch_field_advance_batch(const FieldArgs *descs, const int4 *items, int n_items, bool fold, bool bh,
                                int tile, int halo, hipStream_t s)
{
    FieldLaunch L{nullptr, descs, items, n_items, bh, s};
    field_dispatch(L, fold, tile, halo);
}

}  // namespace pic

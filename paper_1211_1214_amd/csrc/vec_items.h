// Work-item mapping and partial sums shared by the site-parallel kernels.
//
// Workgroups are numbered tile-major / RHS-minor and remapped so that each of the 8 XCDs
// (which receive workgroups round-robin) sweeps one contiguous range: the RHS of a tile
// share its links and clover in that XCD's L2, and neighbouring tiles stay in one L2.
#pragma once
#include "ddwc_internal.h"

namespace ddwc {

__device__ __forceinline__ int xcd_remap(int i, int n) {
    if ((n & 7) != 0) return i;
    return (i & 7) * (n >> 3) + (i >> 3);
}

struct TileRhs {
    int tile, rhs;
};

__device__ __forceinline__ TileRhs tile_rhs(int ntiles, int nrhs) {
    int L = xcd_remap(blockIdx.x, ntiles * nrhs);
    TileRhs t;
    t.tile = L / nrhs;
    t.rhs = L - t.tile * nrhs;
    return t;
}

template <int NV>
__device__ __forceinline__ void write_partials(double v[NV], double* part, int ntiles, TileRhs tr) {
    __shared__ double lds[NV * 16];
    block_sum<NV>(v, lds);
    if (threadIdx.x == 0) {
        double* p = part + ((size_t)tr.rhs * ntiles + tr.tile) * NPART;
#pragma unroll
        for (int k = 0; k < NV; ++k) p[k] = v[k];
    }
}

// Work item of a multi-RHS vector kernel over n sites.  RHS-major fields [nrhs][NCW][n]:
// a workgroup holds WG consecutive sites of one RHS (tiles_of(n) tiles per RHS).
// RHS-innermost fields [NCW][n][nrhs] (RI): a workgroup holds WG consecutive (site, RHS)
// pairs, RHS fastest (tiles_of(n * nrhs) tiles in all).
struct VItem {
    unsigned i;   // site
    int r;        // right-hand side
    bool ok;      // inside the field
    int tile;
    unsigned g0;  // first pair of the workgroup (RI)
};

template <bool RI>
__device__ __forceinline__ VItem vitem(unsigned n, int nrhs, int ntiles) {
    VItem it;
    if (!RI) {
        const TileRhs tr = tile_rhs(ntiles, nrhs);
        it.tile = tr.tile;
        it.r = tr.rhs;
        it.i = tr.tile * WG + threadIdx.x;
        it.ok = it.i < n;
        it.g0 = 0;
    } else {
        it.tile = xcd_remap(blockIdx.x, ntiles);
        it.g0 = (unsigned)it.tile * WG;
        const unsigned gi = it.g0 + threadIdx.x;
        it.ok = gi < n * (unsigned)nrhs;
        it.i = gi / (unsigned)nrhs;
        it.r = (int)(gi - it.i * (unsigned)nrhs);
    }
    return it;
}

// Component stride, element index and base offset (in words) of (site i, RHS r).
template <bool RI, class R>
struct VView {
    unsigned stride, idx;
    size_t base;
    __device__ __forceinline__ VView(unsigned n, int nrhs, unsigned i, int r) {
        if (RI) {
            stride = n * (unsigned)nrhs;
            idx = i * (unsigned)nrhs + r;
            base = 0;
        } else {
            stride = n;
            idx = i;
            base = (size_t)r * Traits<R>::NCW * n;
        }
    }
};

template <int NV, bool RI>
__device__ __forceinline__ void vpartials(double v[NV], double* part, int ntiles, const VItem& it, int nrhs) {
    if (RI) {
        seg_partials<NV>(v, part, ntiles, it.tile, it.g0, nrhs, NPART);
    } else {
        TileRhs tr;
        tr.tile = it.tile;
        tr.rhs = it.r;
        write_partials<NV>(v, part, ntiles, tr);
    }
}

}  // namespace ddwc

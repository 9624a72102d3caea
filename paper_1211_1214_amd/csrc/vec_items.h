// Work-item mapping and partial sums shared by the site-parallel kernels.
//
// Workgroups are numbered tile-major / RHS-minor and remapped so that each of the 8 XCDs
// (which receive workgroups round-robin) sweeps one contiguous range: the RHS of a tile
// share its links and clover in that XCD's L2, and neighbouring tiles stay in one L2.
#pragma once
#include <type_traits>

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

// Partial sums are stored component-major: value k of (RHS r, tile w) at
// part[(k * nrhs + r) * ntiles + w], so that a reduction over the tiles reads each component it
// needs as one contiguous run.
template <int NV>
__device__ __forceinline__ void write_partials(double v[NV], double* part, int ntiles, int nrhs, TileRhs tr) {
    __shared__ double lds[NV * 16];
    block_sum<NV>(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) part[((size_t)k * nrhs + tr.rhs) * ntiles + tr.tile] = v[k];
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

// NT: threads per workgroup of an RHS-innermost kernel (the RHS-major path always uses WG).
// order (RI, may be null): the tile each dispatch slot processes, after the XCD remap.
template <bool RI, int NT = WG>
__device__ __forceinline__ VItem vitem(unsigned n, int nrhs, int ntiles, const int* __restrict__ order = nullptr) {
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
        if (order) it.tile = order[it.tile];
        it.g0 = (unsigned)it.tile * NT;
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

template <int NV, bool RI, int NT = WG, class T = double>
__device__ __forceinline__ void vpartials(double v[NV], double* part, int ntiles, const VItem& it, int nrhs) {
    if (RI) {
        seg_partials<NV, NT, T>(v, part, ntiles, it.tile, it.g0, nrhs);
    } else {
        TileRhs tr;
        tr.tile = it.tile;
        tr.rhs = it.r;
        write_partials<NV>(v, part, ntiles, nrhs, tr);
    }
}

// Staging of what the lanes of one site share (RHS-innermost kernels with at least STG_MIN_RHS
// RHS): the own-site link records, the clover words and the neighbour-table entries of the sites
// a workgroup covers are copied into LDS with coalesced loads before the hop loop, which then
// reads them there: one copy per site instead of one vector-memory load per (site, RHS) lane.
constexpr int STG_MIN_RHS = 8;
template <int NT = WG>
constexpr int stg_sites() {  // sites that NT consecutive (site, RHS) pairs can touch
    return NT / STG_MIN_RHS + 2;
}

template <class S>
constexpr unsigned record_words() {  // 16-byte words of one own-site link record
    return 8 * 9 * sizeof(cx<typename Traits<S>::link>) / 16;
}
template <class S, int NT = WG>
constexpr size_t stage_bytes() {
    return (size_t)stg_sites<NT>() * ((record_words<S>() + Traits<S>::NKW) * 16 + 8 * sizeof(int));
}

// Staging applies to the RHS-innermost low-precision kernels (own-site link records) with enough
// RHS per site.
template <class S>
inline bool stage_ok(int nrhs) {
    return !std::is_same<S, double>::value && nrhs >= STG_MIN_RHS;
}

template <class S>
struct Staged {
    const cx<typename Traits<S>::link>* U;  // link records of sites l0, l0 + 1, ...
    const typename Traits<S>::kword* K;     // clover words [NKW][stg_sites] of the same sites
    const int* nbr;                         // neighbour-table entries [8][stg_sites] of the same sites
    unsigned l0;
};

// Copies the records, clover words and table entries of the sites of the workgroup's pairs;
// every thread of the workgroup must call it (it ends with a barrier).
template <class S, int NT = WG>
__device__ __forceinline__ Staged<S> stage_site_data(const VItem& it, unsigned n2, int nrhs,
                                                     const cx<typename Traits<S>::link>* __restrict__ Up,
                                                     const typename Traits<S>::kword* __restrict__ K,
                                                     const int* __restrict__ nbr) {
    typedef typename Traits<S>::kword KW;
    extern __shared__ float4 stg[];
    constexpr unsigned RW = record_words<S>(), NS = stg_sites<NT>();
    const unsigned l0 = it.g0 / (unsigned)nrhs;
    unsigned l1 = (it.g0 + NT - 1) / (unsigned)nrhs + 1;
    if (l1 > n2) l1 = n2;
    const unsigned ns = l1 - l0;  // <= NS for nrhs >= STG_MIN_RHS
    const float4* src = (const float4*)Up + (size_t)l0 * RW;
    for (unsigned k = threadIdx.x; k < ns * RW; k += NT) stg[k] = src[k];
    KW* ck = (KW*)(stg + NS * RW);
    for (unsigned k = threadIdx.x; k < Traits<S>::NKW * ns; k += NT) {
        const unsigned w = k / ns, j = k - w * ns;
        ck[w * NS + j] = K[(size_t)w * n2 + l0 + j];
    }
    int* cn = (int*)(ck + Traits<S>::NKW * NS);
    for (unsigned k = threadIdx.x; k < 8 * ns; k += NT) {
        const unsigned d = k / ns, j = k - d * ns;
        cn[d * NS + j] = nbr[(size_t)d * n2 + l0 + j];
    }
    __syncthreads();
    Staged<S> st;
    st.U = (const cx<typename Traits<S>::link>*)stg;
    st.K = ck;
    st.nbr = cn;
    st.l0 = l0;
    return st;
}

}  // namespace ddwc

// Site-parallel kernels: layout conversion, clover build, Wilson-clover operator
// variants with fused reductions, BiCGStab vector updates, FP64 reductions.
//
// Mapping: one thread per (site, RHS); a workgroup holds WG consecutive internal
// sites of one RHS.  Workgroups are numbered tile-major / RHS-minor and remapped so
// that each of the 8 XCDs sweeps one contiguous range: the RHS of a tile share its
// links and clover in that XCD's L2, and face neighbours of consecutive Schwarz
// blocks stay in the same L2.
#include <type_traits>

#include <algorithm>

#include "ddwc_internal.h"
#include "clover_build.h"
#include "vec_items.h"

namespace ddwc {

// Operator kernels are memory bound: ask for at least 4 waves per SIMD (<= 128 VGPRs).
#define DDWC_OCC

// ------------------------------------------------------------------ conversions
__global__ void k_links_import(Geom g, const double2* __restrict__ can, cx<double>* __restrict__ U64,
                               cx<float>* __restrict__ U32) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    int mu = blockIdx.y;
    if (s >= g.V) return;
    Site S = decode(g, s);
    int x = canonical_index(g, S);
    const double2* src = can + ((size_t)mu * g.V + x) * 9;
    for (int k = 0; k < 9; ++k) {
        double2 w = src[k];
        size_t o = ((size_t)mu * 9 + k) * g.V + s;
        U64[o] = mk(w.x, w.y);
        U32[o] = mk((float)w.x, (float)w.y);
    }
}

void launch_links_import(Exec& e, const Geom& g, const void* canon, cx<double>* U64, cx<float>* U32) {
    Timed t(e, 4, 0);
    dim3 grid(tiles_of(g.V), 4);
    k_links_import<<<grid, WG, 0, e.stream>>>(g, (const double2*)canon, U64, U32);
}

// Own-site link records [n][8][9] (LK_OWN) of n sites: hop d = 2 mu takes U_mu(x), the site's own
// forward link from Uf ([4][9][n]); d = 2 mu + 1 takes U_mu(x - mu), the forward link of the
// neighbour from Ub ([4][9][*], index from the table nbr [8][n]; the time-boundary sign stays with
// the table entry).  Full lattice: Uf = Ub, one table; even-odd: the two parities' half fields.
__global__ void k_links_own(unsigned n, const cx<float>* __restrict__ Uf, const cx<float>* __restrict__ Ub,
                            unsigned nb, const int* __restrict__ nbr, cx<float>* __restrict__ Lown) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int d = 0; d < 8; ++d) {
        const int mu = d >> 1;
        if (d & 1) {
            const int e = nbr[(size_t)d * n + i];
            const unsigned t = e < 0 ? (unsigned)~e : (unsigned)e;
            for (int k = 0; k < 9; ++k) Lown[(i * 8 + d) * 9 + k] = Ub[((size_t)mu * 9 + k) * nb + t];
        } else {
            for (int k = 0; k < 9; ++k) Lown[(i * 8 + d) * 9 + k] = Uf[((size_t)mu * 9 + k) * n + i];
        }
    }
}

void launch_links_own(Exec& e, unsigned n, const cx<float>* Uf, const cx<float>* Ub, const int* nbr,
                      cx<float>* Lown) {
    Timed t(e, 4, 0);
    k_links_own<<<(unsigned)((n + 255) / 256), 256, 0, e.stream>>>(n, Uf, Ub, n, nbr, Lown);
}

// Neighbour table [8][V] (setup, once per geometry).
__global__ void k_nbr_build(Geom g, int* __restrict__ nbr) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    const Site S = decode(g, s);
    for (int mu = 0; mu < 4; ++mu) {
        nbr[(size_t)(2 * mu) * g.V + s] = table_entry<+1>(g, s, S, mu);
        nbr[(size_t)(2 * mu + 1) * g.V + s] = table_entry<-1>(g, s, S, mu);
    }
}

void launch_nbr_build(Exec& e, const Geom& g, int* nbr) {
    Timed t(e, 4, 0);
    k_nbr_build<<<tiles_of(g.V), WG, 0, e.stream>>>(g, nbr);
}

// Clover term at every site (setup, once per gauge field).
__global__ void k_clover_build(Geom g, const cx<double>* __restrict__ U, double csw, double2* __restrict__ K64,
                               float4* __restrict__ K32) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    double a[72];
    clover_site(g, U, csw, s, a);
    for (int k = 0; k < 36; ++k) K64[(size_t)k * g.V + s] = make_double2(a[2 * k], a[2 * k + 1]);
    for (int k = 0; k < 18; ++k)
        K32[(size_t)k * g.V + s] = make_float4((float)a[4 * k], (float)a[4 * k + 1], (float)a[4 * k + 2], (float)a[4 * k + 3]);
}

void launch_clover_build(Exec& e, const Geom& g, const cx<double>* U64, double csw, double2* K64, float4* K32) {
    Timed t(e, 4, 0);
    k_clover_build<<<(g.V + 127) / 128, 128, 0, e.stream>>>(g, U64, csw, K64, K32);
}

__device__ __forceinline__ bool mask_keep(const Geom& g, const Site& S, int mask) {
    switch (mask) {
        case MASK_P: return in_P(g, S);
        case MASK_BLACK: return S.c == 0;
        case MASK_WHITE: return S.c == 1;
        default: return true;
    }
}

template <class R>
__global__ void k_import(Geom g, const double2* __restrict__ can, typename Traits<R>::word* __restrict__ out,
                         int nrhs, int mask) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    int rhs = blockIdx.y;
    if (s >= g.V) return;
    Site S = decode(g, s);
    bool keep = mask_keep(g, S, mask);
    const double2* src = can + ((size_t)rhs * g.V + canonical_index(g, S)) * 12;
    cx<R> p[12];
    for (int c = 0; c < 12; ++c) {
        double2 w = src[c];
        p[c] = keep ? mk((R)w.x, (R)w.y) : mk(R(0), R(0));
    }
    store_spinor(out + (size_t)rhs * Traits<R>::NCW * g.V, g.V, s, p);
}

template <class R>
__global__ void k_export(Geom g, const typename Traits<R>::word* __restrict__ in, double2* __restrict__ can, int nrhs,
                         int mask) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    int rhs = blockIdx.y;
    if (s >= g.V) return;
    Site S = decode(g, s);
    bool keep = mask_keep(g, S, mask);
    cx<R> p[12];
    load_spinor(in + (size_t)rhs * Traits<R>::NCW * g.V, g.V, s, p);
    double2* dst = can + ((size_t)rhs * g.V + canonical_index(g, S)) * 12;
    for (int c = 0; c < 12; ++c) dst[c] = keep ? make_double2((double)p[c].re, (double)p[c].im) : make_double2(0, 0);
}

template <class R>
void launch_import(Exec& e, const Geom& g, const void* canon, typename Traits<R>::word* out, int nrhs, int mask) {
    Timed t(e, 4, 0);
    k_import<R><<<dim3(tiles_of(g.V), nrhs), WG, 0, e.stream>>>(g, (const double2*)canon, out, nrhs, mask);
}
template <class R>
void launch_export(Exec& e, const Geom& g, const typename Traits<R>::word* in, void* canon, int nrhs, int mask) {
    Timed t(e, 4, 0);
    k_export<R><<<dim3(tiles_of(g.V), nrhs), WG, 0, e.stream>>>(g, in, (double2*)canon, nrhs, mask);
}

// ------------------------------------------------------------------ operator kernels
// Epilogues: DOT partial (aux, y); DOT4 partials (y, in), (y, y), (aux, in), (aux, y) (the global
// BiCGStab's t = M s with aux = rh); RESID: y = aux - y and partial ||y||^2.
enum Epi { EPI_NONE = 0, EPI_DOT = 1, EPI_DOT4 = 2, EPI_RESID = 3 };

template <class R, int EPI>
__global__ __launch_bounds__(WG) DDWC_OCC void k_dslash(Geom g, const cx<R>* __restrict__ U,
                                               const typename Traits<R>::word* __restrict__ K, R mass4,
                                               const typename Traits<R>::word* __restrict__ in,
                                               typename Traits<R>::word* __restrict__ out,
                                               const typename Traits<R>::word* __restrict__ aux, double* part,
                                               int nrhs, int ntiles, const int* __restrict__ nbr, int ndir) {
    typedef typename Traits<R>::word W;
    TileRhs tr = tile_rhs(ntiles, nrhs);
    const int s = tr.tile * WG + threadIdx.x;
    const size_t off = (size_t)tr.rhs * Traits<R>::NCW * g.V;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    if (s < g.V) {
        cx<R> y[12];
        site_operator<R, true, HOPS_ALL, 1>(g, s, in + off, U, K, nbr, mass4, y, ndir);
        if (EPI == EPI_RESID) {
            cx<R> b[12];
            load_spinor((const W*)aux + off, g.V, s, b);
#pragma unroll
            for (int k = 0; k < 12; ++k) y[k] = b[k] - y[k];
            v[0] = acc_nrm(y);
        }
        store_spinor(out + off, g.V, s, y);
        if (EPI == EPI_DOT) {
            cx<R> w[12];
            load_spinor(aux + off, g.V, s, w);
            acc_dot(w, y, v[0], v[1]);
        }
        if (EPI == EPI_DOT4) {
            cx<R> c[12], w[12];
            load_spinor(in + off, g.V, s, c);
            acc_dot(y, c, v[0], v[1]);  // (t, s)
            v[2] = acc_nrm(y);          // (t, t)
            load_spinor(aux + off, g.V, s, w);
            acc_dot(w, c, v[3], v[4]);  // (rh, s)
            acc_dot(w, y, v[5], v[6]);  // (rh, t)
        }
    }
    if (EPI == EPI_DOT) write_partials<2>(v, part, ntiles, nrhs, tr);
    if (EPI == EPI_DOT4) write_partials<7>(v, part, ntiles, nrhs, tr);
    if (EPI == EPI_RESID) write_partials<1>(v, part, ntiles, nrhs, tr);
}

template <class R>
void launch_dslash(Exec& e, const Geom& g, const cx<R>* U, const typename Traits<R>::word* K, double mass4,
                   const typename Traits<R>::word* in, typename Traits<R>::word* out, int nrhs, int kclass,
                   double bytes) {
    Timed t(e, kclass, bytes);
    int nt = tiles_of(g.V);
    k_dslash<R, EPI_NONE><<<nt * nrhs, WG, 0, e.stream>>>(g, U, K, (R)mass4, in, out, nullptr, nullptr, nrhs, nt, e.nbr, 8);
}
template <class R>
void launch_dslash_dot(Exec& e, const Geom& g, const cx<R>* U, const typename Traits<R>::word* K, double mass4,
                       const typename Traits<R>::word* in, typename Traits<R>::word* out,
                       const typename Traits<R>::word* w, double* part, int nrhs, int kclass, double bytes) {
    Timed t(e, kclass, bytes);
    int nt = tiles_of(g.V);
    k_dslash<R, EPI_DOT><<<nt * nrhs, WG, 0, e.stream>>>(g, U, K, (R)mass4, in, out, w, part, nrhs, nt, e.nbr, 8);
}
template <class R>
void launch_dslash_dot4(Exec& e, const Geom& g, const cx<R>* U, const typename Traits<R>::word* K, double mass4,
                        const typename Traits<R>::word* in, typename Traits<R>::word* out,
                        const typename Traits<R>::word* rh, double* part, int nrhs, int kclass, double bytes) {
    Timed t(e, kclass, bytes);
    int nt = tiles_of(g.V);
    k_dslash<R, EPI_DOT4><<<nt * nrhs, WG, 0, e.stream>>>(g, U, K, (R)mass4, in, out, rh, part, nrhs, nt, e.nbr, 8);
}
template <class R>
void launch_residual(Exec& e, const Geom& g, const cx<R>* U, const typename Traits<R>::word* K, double mass4,
                     const typename Traits<R>::word* x, const typename Traits<R>::word* b,
                     typename Traits<R>::word* r, double* part, int nrhs, int kclass, double bytes) {
    Timed t(e, kclass, bytes);
    int nt = tiles_of(g.V);
    k_dslash<R, EPI_RESID><<<nt * nrhs, WG, 0, e.stream>>>(g, U, K, (R)mass4, x, r, b, part, nrhs, nt, e.nbr, 8);
}

template <class R>
__global__ __launch_bounds__(WG) DDWC_OCC void k_hop(Geom g, const cx<R>* __restrict__ U,
                                            const typename Traits<R>::word* __restrict__ in,
                                            typename Traits<R>::word* __restrict__ out, int nrhs, int to_colour,
                                            const int* __restrict__ nbr, int ndir, Ext4 cut, int cut_colour, int s0,
                                            int s1) {
    int s = s0 + blockIdx.x * blockDim.x + threadIdx.x;
    int rhs = blockIdx.y;
    if (s >= s1) return;
    const size_t off = (size_t)rhs * Traits<R>::NCW * g.V;
    cx<R> y[12];
    bool keep = (s / (g.V / 2)) == to_colour;
    if (keep && cut_colour >= 0) {  // output cut to the outer blocks (extents cut) of one colour
        const Site S = decode(g, s);
        int sum = 0;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) sum += (S.n[mu] * g.b[mu] + S.l[mu]) / cut.v[mu];
        keep = (sum & 1) == cut_colour;
    }
    if (keep) {
        // unrolled: 138 VGPRs in FP64 against 256 and AGPRs for the pipelined loop
        site_operator<R, false, HOPS_CROSSING, 2>(g, s, in + off, U, nullptr, nbr, R(0), y, ndir);
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) y[k] = mk(R(0), R(0));
    }
    store_spinor(out + off, g.V, s, y);
}

template <class R>
void launch_hop(Exec& e, const Geom& g, const cx<R>* U, const typename Traits<R>::word* in,
                typename Traits<R>::word* out, int nrhs, int to_colour, const Ext4* cut, int cut_colour,
                bool clear_other) {
    Timed t(e, 4, 0);
    const Ext4 c = cut ? *cut : Ext4{{1, 1, 1, 1}};
    // the sites of colour c are [c V/2, (c + 1) V/2) of the colour-major full index
    const int s0 = clear_other ? 0 : to_colour * (g.V / 2), s1 = clear_other ? g.V : s0 + g.V / 2;
    k_hop<R><<<dim3(tiles_of(s1 - s0), nrhs), WG, 0, e.stream>>>(g, U, in, out, nrhs, to_colour, e.nbr, 8, c,
                                                                 cut ? cut_colour : -1, s0, s1);
}

// ------------------------------------------------------------------ BiCGStab vector kernels
template <class R>
__device__ __forceinline__ cx<R> cxs(const double* a) {
    return mk((R)a[0], (R)a[1]);
}

// Storage S (double, float or H16) with arithmetic in Traits<S>::real; the solution
// correction x is kept in Traits<S>::xs.
#define VTYPES(S)                                       \
    typedef typename Traits<S>::real R;                 \
    typedef typename Traits<S>::xs XS;                  \
    (void)sizeof(R);                                    \
    (void)sizeof(XS)

template <class S, bool RI>
__global__ __launch_bounds__(WG) void k_bicg_init(unsigned n, const double2* __restrict__ r64,
                                                  const double* __restrict__ scale, typename Traits<S>::word* r,
                                                  typename Traits<S>::word* rh, typename Traits<S>::word* p,
                                                  typename Traits<typename Traits<S>::xs>::word* x, double* part,
                                                  int nrhs, int ntiles) {
    VTYPES(S);
    const VItem it = vitem<RI>(n, nrhs, ntiles);
    double v[1] = {0};
    if (it.ok) {
        const VView<RI, S> w(n, nrhs, it.i, it.r);
        const VView<RI, XS> wx(n, nrhs, it.i, it.r);
        cx<double> a[12];
        load_spinor(r64 + (size_t)it.r * 12 * n, n, it.i, a);
        const double sc = scale[it.r];
        cx<R> q[12];
        cx<XS> z[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            q[k] = mk((R)(sc * a[k].re), (R)(sc * a[k].im));
            z[k] = mk(XS(0), XS(0));
        }
        store_spinor(r + w.base, w.stride, w.idx, q);
        store_spinor(rh + w.base, w.stride, w.idx, q);
        store_spinor(p + w.base, w.stride, w.idx, q);
        store_spinor(x + wx.base, wx.stride, wx.idx, z);
        if (std::is_same<S, H16>::value) load_spinor(r + w.base, w.stride, w.idx, q);  // r as stored
        v[0] = acc_nrm(q);
    }
    vpartials<1, RI>(v, part, ntiles, it, nrhs);
}

template <class S, bool RI>
__global__ __launch_bounds__(WG) void k_bicg_s(unsigned n, const BiState* __restrict__ st,
                                               const typename Traits<S>::word* __restrict__ r,
                                               const typename Traits<S>::word* __restrict__ v,
                                               typename Traits<S>::word* __restrict__ s_out, int nrhs, int ntiles) {
    VTYPES(S);
    const VItem it = vitem<RI>(n, nrhs, ntiles);
    if (!it.ok) return;
    const VView<RI, S> w(n, nrhs, it.i, it.r);
    const cx<R> al = cxs<R>(st[it.r].alpha);
    cx<R> a[12], b[12];
    load_spinor(r + w.base, w.stride, w.idx, a);
    load_spinor(v + w.base, w.stride, w.idx, b);
#pragma unroll
    for (int k = 0; k < 12; ++k) a[k] = a[k] - al * b[k];
    store_spinor(s_out + w.base, w.stride, w.idx, a);
}

// x += alpha p + omega s; r = s - omega t; p = r + beta (p - omega v); partial ||r||^2.  beta was
// set from the dot products of t = M s (ST_OMEGA), so the three updates share one pass.
template <class S, bool RI>
__global__ __launch_bounds__(WG) void k_bicg_xrp(unsigned n, const BiState* __restrict__ st,
                                                 typename Traits<typename Traits<S>::xs>::word* __restrict__ x,
                                                 typename Traits<S>::word* __restrict__ p,
                                                 const typename Traits<S>::word* __restrict__ sv,
                                                 const typename Traits<S>::word* __restrict__ t,
                                                 const typename Traits<S>::word* __restrict__ v,
                                                 typename Traits<S>::word* __restrict__ r, double* part, int nrhs,
                                                 int ntiles) {
    VTYPES(S);
    const VItem it = vitem<RI>(n, nrhs, ntiles);
    double q[1] = {0};
    if (it.ok) {
        const VView<RI, S> w(n, nrhs, it.i, it.r);
        const VView<RI, XS> wx(n, nrhs, it.i, it.r);
        const cx<R> al = cxs<R>(st[it.r].alpha), om = cxs<R>(st[it.r].omega), be = cxs<R>(st[it.r].beta);
        cx<XS> xx[12];
        cx<R> pp[12], ss[12], tt[12];
        load_spinor(x + wx.base, wx.stride, wx.idx, xx);
        load_spinor(p + w.base, w.stride, w.idx, pp);
        load_spinor(sv + w.base, w.stride, w.idx, ss);
        load_spinor(t + w.base, w.stride, w.idx, tt);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const cx<R> d = al * pp[k] + om * ss[k];
            xx[k] = xx[k] + mk((XS)d.re, (XS)d.im);
            ss[k] = ss[k] - om * tt[k];
        }
        store_spinor(x + wx.base, wx.stride, wx.idx, xx);
        store_spinor(r + w.base, w.stride, w.idx, ss);
        if (std::is_same<S, H16>::value) load_spinor(r + w.base, w.stride, w.idx, ss);  // r as stored
        q[0] = acc_nrm(ss);
        load_spinor(v + w.base, w.stride, w.idx, tt);
#pragma unroll
        for (int k = 0; k < 12; ++k) pp[k] = ss[k] + be * (pp[k] - om * tt[k]);
        store_spinor(p + w.base, w.stride, w.idx, pp);
    }
    vpartials<1, RI>(q, part, ntiles, it, nrhs);
}

template <class S, bool RI>
__global__ __launch_bounds__(WG) void k_accumulate(unsigned n,
                                                   const typename Traits<typename Traits<S>::xs>::word* __restrict__ x,
                                                   const double* __restrict__ scale, double2* __restrict__ x64,
                                                   int nrhs, int ntiles) {
    VTYPES(S);
    const VItem it = vitem<RI>(n, nrhs, ntiles);
    if (!it.ok) return;
    const double sc = scale[it.r];
    if (sc == 0.0) return;
    const double inv = 1.0 / sc;
    const VView<RI, XS> wx(n, nrhs, it.i, it.r);
    cx<XS> a[12];
    cx<double> b[12];
    load_spinor(x + wx.base, wx.stride, wx.idx, a);
    double2* dst = x64 + (size_t)it.r * 12 * n;
    load_spinor(dst, n, it.i, b);
#pragma unroll
    for (int k = 0; k < 12; ++k) b[k] = b[k] + mk(inv * (double)a[k].re, inv * (double)a[k].im);
    store_spinor(dst, n, it.i, b);
}
#undef VTYPES

int vector_tiles(unsigned n, int nrhs, bool ri) { return ri ? tiles_of((int)(n * (unsigned)nrhs)) : tiles_of((int)n); }
static int vector_grid(unsigned n, int nrhs, bool ri) { return ri ? vector_tiles(n, nrhs, ri) : tiles_of((int)n) * nrhs; }

#define VDISPATCH(KERNEL, S, ...)                                                                          \
    do {                                                                                                   \
        const int nt = vector_tiles(n, nrhs, ri), ng = vector_grid(n, nrhs, ri);                           \
        if (ri)                                                                                            \
            KERNEL<S, true><<<ng, WG, 0, e.stream>>>(n, __VA_ARGS__, nrhs, nt);                             \
        else                                                                                               \
            KERNEL<S, false><<<ng, WG, 0, e.stream>>>(n, __VA_ARGS__, nrhs, nt);                            \
    } while (0)

template <class S>
void launch_bicg_init(Exec& e, unsigned n, bool ri, const double2* r64, const double* scale,
                      typename Traits<S>::word* r, typename Traits<S>::word* rh, typename Traits<S>::word* p,
                      typename Traits<typename Traits<S>::xs>::word* x, double* part, int nrhs) {
    Timed t(e, 3, 0);
    VDISPATCH(k_bicg_init, S, r64, scale, r, rh, p, x, part);
}
template <class S>
void launch_bicg_s(Exec& e, unsigned n, bool ri, const BiState* st, const typename Traits<S>::word* r,
                   const typename Traits<S>::word* v, typename Traits<S>::word* s, int nrhs) {
    Timed t(e, 3, 0);
    VDISPATCH(k_bicg_s, S, st, r, v, s);
}
template <class S>
void launch_bicg_xrp(Exec& e, unsigned n, bool ri, const BiState* st, typename Traits<typename Traits<S>::xs>::word* x,
                     typename Traits<S>::word* p, const typename Traits<S>::word* s, const typename Traits<S>::word* t,
                     const typename Traits<S>::word* v, typename Traits<S>::word* r, double* part, int nrhs) {
    Timed tm(e, 3, 0);
    VDISPATCH(k_bicg_xrp, S, st, x, p, s, t, v, r, part);
}
template <class S>
void launch_accumulate(Exec& e, unsigned n, bool ri, const typename Traits<typename Traits<S>::xs>::word* x,
                       const double* scale, double2* x64, int nrhs) {
    Timed t(e, 3, 0);
    VDISPATCH(k_accumulate, S, x, scale, x64);
}
#undef VDISPATCH

// ------------------------------------------------------------------ reproducible test data
// v[i] = (u(2i), u(2i + 1)) - 1/2 with u a 64-bit integer hash mapped to [0, 1) (the
// SplitMix64 finaliser); used by the autotuner for its right-hand sides.
__device__ __forceinline__ double hash_unit(uint64_t z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}
__global__ void k_fill_hash(double2* __restrict__ v, size_t n, uint64_t seed) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    v[i] = make_double2(hash_unit(seed + 2 * i) - 0.5, hash_unit(seed + 2 * i + 1) - 0.5);
}
void launch_fill_hash(Exec& e, double2* v, size_t n, uint64_t seed) {
    Timed t(e, 4, 0);
    k_fill_hash<<<(unsigned)((n + 255) / 256), 256, 0, e.stream>>>(v, n, seed);
}

// ------------------------------------------------------------------ streaming reference
// dst = src over n 16-byte words: the streaming rate the operator kernels are measured against
// (and a transfer of known size for calibrating memory counters).  Each thread moves eight words
// per round, all eight loads issued before the stores (non-temporal: the data is not reused);
// rounds stride over the whole grid.
typedef float v4f __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_stream_copy(const v4f* __restrict__ src, v4f* __restrict__ dst, size_t n) {
    constexpr int U = 8;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (U - 1) * stride < n; i += U * stride) {
        v4f w[U];
#pragma unroll
        for (int k = 0; k < U; ++k) w[k] = __builtin_nontemporal_load(src + i + k * stride);
#pragma unroll
        for (int k = 0; k < U; ++k) __builtin_nontemporal_store(w[k], dst + i + k * stride);
    }
    for (; i < n; i += stride) dst[i] = src[i];
}
void launch_stream_copy(Exec& e, const float4* src, float4* dst, size_t n) {
    const size_t want = (n + 2047) / 2048;  // eight words per thread and round
    const unsigned grid = (unsigned)std::min<size_t>(std::max<size_t>(want, 1), 8192);
    k_stream_copy<<<grid, 256, 0, e.stream>>>((const v4f*)src, (v4f*)dst, n);
}

// ------------------------------------------------------------------ finalize (one workgroup per RHS)
// Sums the first NV partial components of each RHS over the tiles (fixed order), then applies
// the BiCGStab stage.  v has NPART entries so that every stage can name its components.
template <int NV>
__global__ __launch_bounds__(1024) void k_finalize(const double* __restrict__ part, int ntiles, int nrhs,
                                                  double* __restrict__ sums, BiState* __restrict__ st, int stage,
                                                  const double* __restrict__ thr_rel2) {
    const int rhs = blockIdx.x;
    double v[NPART] = {};
    // four strides in flight per thread (independent sums, combined in a fixed order): a single
    // workgroup per RHS is otherwise bound by the latency of one load round per stride
    constexpr int U = 4;
    double a[U][NV] = {};
    const unsigned B = blockDim.x;
    unsigned w = threadIdx.x;
    for (; w + (U - 1) * B < (unsigned)ntiles; w += U * B) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < NV; ++k) a[u][k] += part[((size_t)k * nrhs + rhs) * ntiles + w + u * B];
    }
    for (; w < (unsigned)ntiles; w += B) {
#pragma unroll
        for (int k = 0; k < NV; ++k) a[0][k] += part[((size_t)k * nrhs + rhs) * ntiles + w];
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = (a[0][k] + a[1][k]) + (a[2][k] + a[3][k]);
    __shared__ double lds[NV * 16];
    block_sum<NV>(v, lds);
    if (threadIdx.x != 0) return;
    if (sums)
        for (int k = 0; k < NV; ++k) sums[rhs * NPART + k] = v[k];
    if (!st) return;
    BiState S = st[rhs];
    if (stage == ST_INIT) {
        S.rho[0] = v[0];
        S.rho[1] = 0;
        S.rr = v[0];
        S.thr2 = thr_rel2[rhs] * v[0];
        S.active = (v[0] > S.thr2 && thr_rel2[rhs] < 1.0) ? 1 : 0;
        S.broken = 0;
        S.alpha[0] = S.alpha[1] = S.omega[0] = S.omega[1] = S.beta[0] = S.beta[1] = 0;
    } else if (stage == ST_ALPHA) {
        double d = v[0] * v[0] + v[1] * v[1];
        if (S.active && d > 0 && isfinite(d)) {
            // alpha = rho / (rh, v)
            S.alpha[0] = (S.rho[0] * v[0] + S.rho[1] * v[1]) / d;
            S.alpha[1] = (S.rho[1] * v[0] - S.rho[0] * v[1]) / d;
        } else {
            if (S.active) S.broken = 1;
            S.active = 0;
            S.alpha[0] = S.alpha[1] = 0;
        }
    } else if (stage == ST_OMEGA) {
        // v: (t, s), (t, t), (rh, s), (rh, t).  omega = (t, s) / (t, t); the next rho is
        // (rh, s - omega t) = (rh, s) - omega (rh, t); beta = (rho_next / rho) (alpha / omega).
        S.beta[0] = S.beta[1] = 0;
        if (S.active && v[2] > 0 && isfinite(v[2])) {
            S.omega[0] = v[0] / v[2];
            S.omega[1] = v[1] / v[2];
            const double nr = v[3] - (S.omega[0] * v[5] - S.omega[1] * v[6]);
            const double ni = v[4] - (S.omega[0] * v[6] + S.omega[1] * v[5]);
            const double om2 = S.omega[0] * S.omega[0] + S.omega[1] * S.omega[1];
            const double rh2 = S.rho[0] * S.rho[0] + S.rho[1] * S.rho[1];
            if (om2 > 0 && rh2 > 0) {
                const double qr = (nr * S.rho[0] + ni * S.rho[1]) / rh2;
                const double qi = (ni * S.rho[0] - nr * S.rho[1]) / rh2;
                const double ar = (S.alpha[0] * S.omega[0] + S.alpha[1] * S.omega[1]) / om2;
                const double ai = (S.alpha[1] * S.omega[0] - S.alpha[0] * S.omega[1]) / om2;
                S.beta[0] = qr * ar - qi * ai;
                S.beta[1] = qr * ai + qi * ar;
            }
            S.rho[0] = nr;
            S.rho[1] = ni;
        } else {
            // t = 0 means s = 0: x += alpha p is exact, and ST_RR stops here
            S.omega[0] = S.omega[1] = 0;
            if (S.active && !(v[2] >= 0)) S.broken = 1;
        }
    } else if (stage == ST_RR) {
        if (S.active) {
            S.rr = v[0];
            const double om2 = S.omega[0] * S.omega[0] + S.omega[1] * S.omega[1];
            const double rh2 = S.rho[0] * S.rho[0] + S.rho[1] * S.rho[1];
            if (!isfinite(v[0])) {
                S.broken = 1;
                S.active = 0;
            } else if (v[0] <= S.thr2) {
                S.active = 0;
            } else if (om2 == 0 || rh2 == 0) {
                S.broken = 1;
                S.active = 0;
            }
        }
        if (!S.active) {
            S.alpha[0] = S.alpha[1] = S.omega[0] = S.omega[1] = S.beta[0] = S.beta[1] = 0;
        }
    }
    st[rhs] = S;
}

void launch_finalize(Exec& e, const double* part, int ntiles, int nrhs, double* sums, BiState* st, int stage,
                     const double* thr_rel2, int nv) {
    Timed t(e, 3, 0);
    if (nv < 0) nv = stage == ST_ALPHA ? 2 : stage == ST_OMEGA ? 7 : stage == ST_SUM ? 3 : 1;
    // one workgroup of 16 waves per RHS: the partial sums of up to ~10^4 tiles in a few strides
#define FIN(N) k_finalize<N><<<nrhs, 1024, 0, e.stream>>>(part, ntiles, nrhs, sums, st, stage, thr_rel2)
    switch (nv) {
        case 1: FIN(1); break;
        case 2: FIN(2); break;
        case 3: FIN(3); break;
        default: FIN(7); break;
    }
#undef FIN
}

// ------------------------------------------------------------------ FP64 helpers
__global__ __launch_bounds__(WG) void k_axpby(Geom g, double a, const double2* __restrict__ x, double b,
                                              const double2* __restrict__ y, double2* __restrict__ z, int nrhs,
                                              int mask) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    int rhs = blockIdx.y;
    if (s >= g.V) return;
    Site S = decode(g, s);
    bool keep = mask_keep(g, S, mask);
    const size_t off = (size_t)rhs * 12 * g.V;
    cx<double> u[12], w[12];
    for (int k = 0; k < 12; ++k) u[k] = w[k] = mk(0.0, 0.0);
    if (keep) {
        if (x) load_spinor(x + off, g.V, s, u);
        if (y) load_spinor(y + off, g.V, s, w);
        for (int k = 0; k < 12; ++k) u[k] = a * u[k] + b * w[k];
    }
    store_spinor(z + off, g.V, s, u);
}

void launch_axpby(Exec& e, const Geom& g, double a, const double2* x, double b, const double2* y, double2* z,
                  int nrhs, int mask) {
    Timed t(e, 4, 0);
    k_axpby<<<dim3(tiles_of(g.V), nrhs), WG, 0, e.stream>>>(g, a, x, b, y, z, nrhs, mask);
}

// y = y + c_r x for every RHS r, c device [nrhs] complex (GCR updates); no site mask.
__global__ __launch_bounds__(WG) void k_caxpy(unsigned V, const double2* __restrict__ c, const double2* __restrict__ x,
                                              double2* __restrict__ y) {
    const unsigned s = blockIdx.x * blockDim.x + threadIdx.x;
    const int rhs = blockIdx.y;
    if (s >= V) return;
    const double2 cw = c[rhs];
    if (cw.x == 0.0 && cw.y == 0.0) return;
    const cx<double> cc = mk(cw.x, cw.y);
    const size_t off = (size_t)rhs * 12 * V;
    cx<double> u[12], w[12];
    load_spinor(x + off, V, s, u);
    load_spinor(y + off, V, s, w);
#pragma unroll
    for (int k = 0; k < 12; ++k) w[k] = w[k] + cc * u[k];
    store_spinor(y + off, V, s, w);
}

void launch_caxpy(Exec& e, const Geom& g, const double2* c, const double2* x, double2* y, int nrhs) {
    Timed t(e, 3, 0);
    k_caxpy<<<dim3(tiles_of(g.V), nrhs), WG, 0, e.stream>>>((unsigned)g.V, c, x, y);
}

// ------------------------------------------------------------------ nested domain decomposition
// v = 0 at every site outside the outer Schwarz blocks of one colour (outer extents Bo): the
// cut that turns a hop of the inner decomposition into a hop of the Dirichlet operator of
// those outer blocks.
__global__ __launch_bounds__(WG) void k_region(Geom g, Ext4 Bo, int colour, double2* __restrict__ v, int nrhs) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int rhs = blockIdx.y;
    if (s >= g.V) return;
    const Site S = decode(g, s);
    int sum = 0;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) sum += (S.n[mu] * g.b[mu] + S.l[mu]) / Bo.v[mu];
    if ((sum & 1) == colour) return;
    double2* f = v + (size_t)rhs * 12 * g.V;
#pragma unroll
    for (int c = 0; c < 12; ++c) f[(size_t)c * g.V + s] = make_double2(0.0, 0.0);
}

void launch_region(Exec& e, const Geom& g, const Ext4& Bo, int colour, double2* v, int nrhs) {
    Timed t(e, 4, 0);
    k_region<<<dim3(tiles_of(g.V), nrhs), WG, 0, e.stream>>>(g, Bo, colour, v, nrhs);
}

// dst (internal order of gd) = src (internal order of gs): the same lattice under two block sizes.
__global__ __launch_bounds__(WG) void k_relayout(Geom gs, Geom gd, const double2* __restrict__ src,
                                                 double2* __restrict__ dst, int nrhs) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int rhs = blockIdx.y;
    if (s >= gd.V) return;
    const Site S = decode(gd, s);
    int n[4], l[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const int x = S.n[mu] * gd.b[mu] + S.l[mu];
        n[mu] = x / gs.b[mu];
        l[mu] = x % gs.b[mu];
    }
    const int t = block_base(gs, n) + local_index(gs, l);
    const size_t off = (size_t)rhs * 12 * gd.V;
#pragma unroll
    for (int c = 0; c < 12; ++c) dst[off + (size_t)c * gd.V + s] = src[off + (size_t)c * gd.V + t];
}

void launch_relayout(Exec& e, const Geom& gs, const Geom& gd, const double2* src, double2* dst, int nrhs) {
    Timed t(e, 4, 0);
    k_relayout<<<dim3(tiles_of(gd.V), nrhs), WG, 0, e.stream>>>(gs, gd, src, dst, nrhs);
}

// Fingerprint of canonical links (n complex numbers): sum_i Re u_i h(2i) + Im u_i h(2i + 1) with
// hash weights, in a fixed order (FP_BLOCKS workgroup partials, summed on the host in order), so
// that equal link arrays give bit-equal fingerprints.
__global__ __launch_bounds__(256) void k_link_fp(const double2* __restrict__ u, size_t n, double* __restrict__ part) {
    double v[1] = {0.0};
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)FP_BLOCKS * 256) {
        const double2 w = u[i];
        v[0] += w.x * (hash_unit(2 * i) - 0.5) + w.y * (hash_unit(2 * i + 1) - 0.5);
    }
    __shared__ double lds[16];
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

void launch_link_fp(Exec& e, const void* links, size_t n, double* part) {
    Timed t(e, 4, 0);
    k_link_fp<<<FP_BLOCKS, 256, 0, e.stream>>>((const double2*)links, n, part);
}

__global__ __launch_bounds__(WG) void k_dots(Geom g, const double2* __restrict__ x, const double2* __restrict__ y,
                                             double* part, int nrhs, int ntiles) {
    TileRhs tr = tile_rhs(ntiles, nrhs);
    const int s = tr.tile * WG + threadIdx.x;
    double v[3] = {0, 0, 0};
    if (s < g.V) {
        const size_t off = (size_t)tr.rhs * 12 * g.V;
        cx<double> a[12], b[12];
        load_spinor(x + off, g.V, s, a);
        load_spinor(y + off, g.V, s, b);
        acc_dot(a, b, v[0], v[1]);
        v[2] = acc_nrm(b);
    }
    write_partials<3>(v, part, ntiles, nrhs, tr);
}

void launch_dots(Exec& e, const Geom& g, const double2* x, const double2* y, double* part, int nrhs) {
    Timed t(e, 3, 0);
    int nt = tiles_of(g.V);
    k_dots<<<nt * nrhs, WG, 0, e.stream>>>(g, x, y, part, nrhs, nt);
}

// ------------------------------------------------------------------ RHS-innermost FP32 full Dslash
// Fields [6][V][nrhs] float4 (vec_items.h), site-major FP32 links [V][4][9]: the lanes of a site
// (its RHS) share one link record and one clover load, as in the global solver's kernels.
__global__ __launch_bounds__(WG) void k_import_ri32(Geom g, const double2* __restrict__ can, float4* __restrict__ out,
                                                    int nrhs, int ntiles) {
    const VItem it = vitem<true>((unsigned)g.V, nrhs, ntiles);
    if (!it.ok) return;
    const VView<true, float> w((unsigned)g.V, nrhs, it.i, it.r);
    const double2* src = can + ((size_t)it.r * g.V + canonical_index(g, decode(g, (int)it.i))) * 12;
    cx<float> q[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const double2 v = src[c];
        q[c] = mk((float)v.x, (float)v.y);
    }
    store_spinor(out, w.stride, w.idx, q);
}

__global__ __launch_bounds__(WG) void k_export_ri32(Geom g, const float4* __restrict__ in, double2* __restrict__ can,
                                                    int nrhs, int ntiles) {
    const VItem it = vitem<true>((unsigned)g.V, nrhs, ntiles);
    if (!it.ok) return;
    const VView<true, float> w((unsigned)g.V, nrhs, it.i, it.r);
    cx<float> q[12];
    load_spinor(in, w.stride, w.idx, q);
    double2* dst = can + ((size_t)it.r * g.V + canonical_index(g, decode(g, (int)it.i))) * 12;
#pragma unroll
    for (int c = 0; c < 12; ++c) dst[c] = make_double2((double)q[c].re, (double)q[c].im);
}

// NT threads per workgroup; order (may be null): the tile of each dispatch slot.
template <bool STG, int NT>
__global__ __launch_bounds__(NT) void k_dslash_ri32(Geom g, const cx<float>* __restrict__ Lown,
                                                    const float4* __restrict__ K, float mass4,
                                                    const float4* __restrict__ in, float4* __restrict__ out,
                                                    const int* __restrict__ nbr, int nrhs, int ntiles,
                                                    const int* __restrict__ order) {
    const VItem it = vitem<true, NT>((unsigned)g.V, nrhs, ntiles, order);
    const cx<float>* Uf = Lown;
    const float4* Kk = K;
    const int* nb = nbr;
    unsigned kst = (unsigned)g.V, l0 = 0, nstr = 0;
    if (STG) {
        const Staged<float> sd = stage_site_data<float, NT>(it, (unsigned)g.V, nrhs, Lown, K, nbr);
        Uf = sd.U;
        Kk = sd.K;
        nb = sd.nbr;
        kst = nstr = stg_sites<NT>();
        l0 = sd.l0;
    }
    if (!it.ok) return;
    const VView<true, float> w((unsigned)g.V, nrhs, it.i, it.r);
    cx<float> acc[12], c[12];
    hop_sum<float, HOPS_ALL, STG ? 0 : 1, LK_OWN>((unsigned)g.V, it.i, in, Uf, Uf, nb, acc, 8, (unsigned)nrhs,
                                                  (unsigned)it.r, w.stride, l0, nstr);
    load_spinor(in, w.stride, w.idx, c);
    apply_diag<float>(Kk, kst, it.i - l0, mass4, c, acc, -0.5f);
    store_spinor(out, w.stride, w.idx, acc);
}

void launch_import_ri32(Exec& e, const Geom& g, const void* canon, float4* out, int nrhs) {
    Timed t(e, 4, 0);
    const int nt = tiles_of(g.V * nrhs);
    k_import_ri32<<<nt, WG, 0, e.stream>>>(g, (const double2*)canon, out, nrhs, nt);
}
void launch_export_ri32(Exec& e, const Geom& g, const float4* in, void* canon, int nrhs) {
    Timed t(e, 4, 0);
    const int nt = tiles_of(g.V * nrhs);
    k_export_ri32<<<nt, WG, 0, e.stream>>>(g, in, (double2*)canon, nrhs, nt);
}
void launch_dslash_ri32(Exec& e, const Geom& g, const cx<float>* Us, const float4* K, double mass4, const float4* in,
                        float4* out, int nrhs, int kclass, double bytes, int op_threads, const int* order) {
    Timed t(e, kclass, bytes);
    const int NTr = nrhs <= op_threads ? op_threads : WG;
    const int nt = (int)(((long long)g.V * nrhs + NTr - 1) / NTr);
    auto launch = [&](auto ntc) {
        constexpr int NT = decltype(ntc)::value;
        if (stage_ok<float>(nrhs))
            k_dslash_ri32<true, NT><<<nt, NT, stage_bytes<float, NT>(), e.stream>>>(g, Us, K, (float)mass4, in, out,
                                                                                  e.nbr, nrhs, nt, order);
        else
            k_dslash_ri32<false, NT><<<nt, NT, 0, e.stream>>>(g, Us, K, (float)mass4, in, out, e.nbr, nrhs, nt, order);
    };
    switch (NTr) {
        case 128: launch(std::integral_constant<int, 128>()); break;
        case 512: launch(std::integral_constant<int, 512>()); break;
        default: launch(std::integral_constant<int, WG>()); break;
    }
}
int dslash_ri32_tiles(const Geom& g, int nrhs, int op_threads) {
    const int NTr = nrhs <= op_threads ? op_threads : WG;
    return (int)(((long long)g.V * nrhs + NTr - 1) / NTr);
}

// ------------------------------------------------------------------ instantiations
#define INST(R)                                                                                                    \
    template void launch_import<R>(Exec&, const Geom&, const void*, Traits<R>::word*, int, int);                  \
    template void launch_export<R>(Exec&, const Geom&, const Traits<R>::word*, void*, int, int);                  \
    template void launch_dslash<R>(Exec&, const Geom&, const cx<R>*, const Traits<R>::word*, double,              \
                                   const Traits<R>::word*, Traits<R>::word*, int, int, double);                   \
    template void launch_dslash_dot<R>(Exec&, const Geom&, const cx<R>*, const Traits<R>::word*, double,          \
                                       const Traits<R>::word*, Traits<R>::word*, const Traits<R>::word*, double*, \
                                       int, int, double);                                                         \
    template void launch_dslash_dot4<R>(Exec&, const Geom&, const cx<R>*, const Traits<R>::word*, double,         \
                                        const Traits<R>::word*, Traits<R>::word*, const Traits<R>::word*,         \
                                        double*, int, int, double);                                               \
    template void launch_residual<R>(Exec&, const Geom&, const cx<R>*, const Traits<R>::word*, double,            \
                                     const Traits<R>::word*, const Traits<R>::word*, Traits<R>::word*, double*,   \
                                     int, int, double);                                                           \
    template void launch_hop<R>(Exec&, const Geom&, const cx<R>*, const Traits<R>::word*, Traits<R>::word*, int,  \
                                int, const Ext4*, int, bool);                                                     \
    template void launch_bicg_init<R>(Exec&, unsigned, bool, const double2*, const double*, Traits<R>::word*,      \
                                      Traits<R>::word*, Traits<R>::word*, Traits<R>::word*, double*, int);        \
    template void launch_bicg_s<R>(Exec&, unsigned, bool, const BiState*, const Traits<R>::word*,                 \
                                   const Traits<R>::word*, Traits<R>::word*, int);                                \
    template void launch_bicg_xrp<R>(Exec&, unsigned, bool, const BiState*, Traits<R>::word*, Traits<R>::word*,   \
                                     const Traits<R>::word*, const Traits<R>::word*, const Traits<R>::word*,      \
                                     Traits<R>::word*, double*, int);                                             \
    template void launch_accumulate<R>(Exec&, unsigned, bool, const Traits<R>::word*, const double*, double2*, int);

INST(double)
INST(float)

template void launch_bicg_init<H16>(Exec&, unsigned, bool, const double2*, const double*, hw16*, hw16*, hw16*, float4*,
                                    double*, int);
template void launch_bicg_s<H16>(Exec&, unsigned, bool, const BiState*, const hw16*, const hw16*, hw16*, int);
template void launch_bicg_xrp<H16>(Exec&, unsigned, bool, const BiState*, float4*, hw16*, const hw16*, const hw16*,
                                   const hw16*, hw16*, double*, int);
template void launch_accumulate<H16>(Exec&, unsigned, bool, const float4*, const double*, double2*, int);

}  // namespace ddwc

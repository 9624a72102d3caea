// Even-odd preconditioned operator kernels on half fields (see eo.h for the algebra).
#include "ddwc_internal.h"
#include "eo.h"
#include "vec_items.h"

namespace ddwc {

// ------------------------------------------------------------------ setup
__global__ void k_eo_setup(Geom g, const cx<double>* __restrict__ U64, const double2* __restrict__ K64,
                           const int* __restrict__ nbr, cx<double>* __restrict__ Uh64, cx<float>* __restrict__ Uh32,
                           double2* __restrict__ Kh64, float4* __restrict__ Kh32, int* __restrict__ nbr_eo) {
    const unsigned s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= (unsigned)g.V) return;
    const size_t V = g.V, V2 = g.V / 2;
    int p;
    const unsigned i = half_index(g, s, p);
    for (int mu = 0; mu < 4; ++mu)
        for (int k = 0; k < 9; ++k) {
            const cx<double> u = U64[((size_t)mu * 9 + k) * V + s];
            const size_t o = (((size_t)p * 4 + mu) * 9 + k) * V2 + i;
            Uh64[o] = u;
            Uh32[o] = mk((float)u.re, (float)u.im);
        }
    double a[72];
    for (int k = 0; k < 36; ++k) {
        const double2 w = K64[(size_t)k * V + s];
        a[2 * k] = w.x;
        a[2 * k + 1] = w.y;
        Kh64[((size_t)p * 36 + k) * V2 + i] = w;
    }
    for (int k = 0; k < 18; ++k)
        Kh32[((size_t)p * 18 + k) * V2 + i] =
            make_float4((float)a[4 * k], (float)a[4 * k + 1], (float)a[4 * k + 2], (float)a[4 * k + 3]);
    for (int d = 0; d < 8; ++d) nbr_eo[((size_t)p * 8 + d) * V2 + i] = half_entry(g, nbr[(size_t)d * V + s]);
}

void launch_eo_setup(Exec& e, const Geom& g, const cx<double>* U64, const double2* K64, const int* nbr,
                     cx<double>* Uh64, cx<float>* Uh32, double2* Kh64, float4* Kh32, int* nbr_eo) {
    Timed t(e, 4, 0);
    k_eo_setup<<<tiles_of(g.V), WG, 0, e.stream>>>(g, U64, K64, nbr, Uh64, Uh32, Kh64, Kh32, nbr_eo);
}

void launch_eo_links_own(Exec& e, unsigned n2, const cx<float>* Uh32, const int* nbr_eo, cx<float>* Lown) {
    // parity p: forward links of the parity-p sites, backward links from the other parity's
    for (int p = 0; p < 2; ++p)
        launch_links_own(e, n2, Uh32 + (size_t)p * 36 * n2, Uh32 + (size_t)(1 - p) * 36 * n2, nbr_eo + (size_t)p * 8 * n2,
                         Lown + (size_t)p * 72 * n2);
}

// FP16 copy of the FP32 half-order links (setup).
__global__ void k_links_to_half(size_t n, const cx<float>* __restrict__ src, cx<f16>* __restrict__ dst) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const cx<float> v = src[i];
    dst[i] = mk((f16)v.re, (f16)v.im);
}

void launch_links_to_half(Exec& e, size_t n, const cx<float>* src, cx<f16>* dst) {
    Timed t(e, 4, 0);
    k_links_to_half<<<(unsigned)((n + 255) / 256), 256, 0, e.stream>>>(n, src, dst);
}

// A_pp^-1 for the sites of parity p of half clover Kp (once per mass).
__global__ void k_eo_inverse(unsigned V2, const double2* __restrict__ Kp, double mass4, double2* __restrict__ A64,
                             float4* __restrict__ A32) {
    const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V2) return;
    double a[72], b[72];
    for (int k = 0; k < 36; ++k) {
        const double2 w = Kp[(size_t)k * V2 + i];
        a[2 * k] = w.x;
        a[2 * k + 1] = w.y;
    }
    clover_inverse_site(a, mass4, b);
    for (int k = 0; k < 36; ++k) A64[(size_t)k * V2 + i] = make_double2(b[2 * k], b[2 * k + 1]);
    for (int k = 0; k < 18; ++k)
        A32[(size_t)k * V2 + i] = make_float4((float)b[4 * k], (float)b[4 * k + 1], (float)b[4 * k + 2], (float)b[4 * k + 3]);
}

void launch_eo_inverse(Exec& e, unsigned V2, const double2* Kp, double mass4, double2* A64, float4* A32) {
    Timed t(e, 4, 0);
    k_eo_inverse<<<(V2 + 127) / 128, 128, 0, e.stream>>>(V2, Kp, mass4, A64, A32);
}

// full FP64 field <-> (even, odd) FP64 half fields; merging, the odd part is ho + w2 ho2 when
// ho2 is given
__global__ void k_eo_split(Geom g, const double2* __restrict__ full, double2* __restrict__ he, double2* __restrict__ ho,
                           int merge, const double2* __restrict__ ho2, double w2) {
    const unsigned s = blockIdx.x * blockDim.x + threadIdx.x;
    const int rhs = blockIdx.y;
    if (s >= (unsigned)g.V) return;
    const size_t V = g.V, V2 = g.V / 2;
    int p;
    const unsigned i = half_index(g, s, p);
    double2* h = p ? ho : he;
    const bool add = merge && p && ho2;
    for (int c = 0; c < 12; ++c) {
        const size_t hi = ((size_t)rhs * 12 + c) * V2 + i;
        if (merge) {
            double2 v = h[hi];
            if (add) {
                const double2 a = ho2[hi];
                v = make_double2(v.x + w2 * a.x, v.y + w2 * a.y);
            }
            ((double2*)full)[((size_t)rhs * 12 + c) * V + s] = v;
        } else {
            h[hi] = full[((size_t)rhs * 12 + c) * V + s];
        }
    }
}

void launch_eo_split(Exec& e, const Geom& g, const double2* full, double2* he, double2* ho, int nrhs) {
    Timed t(e, 4, 0);
    k_eo_split<<<dim3(tiles_of(g.V), nrhs), WG, 0, e.stream>>>(g, full, he, ho, 0, nullptr, 0.0);
}
void launch_eo_merge(Exec& e, const Geom& g, const double2* he, const double2* ho, double2* full, int nrhs,
                     const double2* ho2, double w2) {
    Timed t(e, 4, 0);
    k_eo_split<<<dim3(tiles_of(g.V), nrhs), WG, 0, e.stream>>>(g, full, (double2*)he, (double2*)ho, 1, ho2, w2);
}

// ------------------------------------------------------------------ operator kernels
// The RHS-innermost FP32/FP16 kernels (the global solver) read own-site link records (each half
// site's eight hop links in one contiguous record); FP64 and the RHS-major kernels read
// entry-major links (EoFields of eo_fields with site_major set alike).
template <class S, bool RI>
constexpr int site_major_links() {
    return RI && !std::is_same<S, double>::value ? LK_OWN : LK_ENTRY;
}

// Pipelining of the hop loop (hop_sum): with the links, clover and table staged in LDS the
// unpipelined loop's fewer registers (about 100 against 146) buy a fourth and fifth wave per
// SIMD, which hides the neighbour-spinor latency better than loading one direction ahead.  (In
// FP64 the pipelined loop needs 254 VGPRs, one wave per SIMD, and is still as fast as the
// unpipelined one at two waves.)
template <bool STG>
constexpr int hop_pipe() {
    return STG ? 0 : 1;
}

// Work items as for the vector kernels (vec_items.h): RHS-major fields or, with RI, the
// RHS-innermost layout in which the lanes of a site share its links, clover and table.

// y_p = A_pp^-1 (c_p + alpha H_{p,1-p} x), over the n2 sites of parity p.  c may be null,
// alpha = 0 skips the hops.  S is the storage (double, float or H16), arithmetic in its real.
template <class S, bool RI, bool STG, int NT>
__global__ __launch_bounds__(NT) void k_eo_hopinv(unsigned n2, const typename Traits<S>::word* __restrict__ x,
                                                  const typename Traits<S>::word* __restrict__ c,
                                                  typename Traits<S>::real alpha,
                                                  const cx<typename Traits<S>::link>* __restrict__ Up,
                                                  const cx<typename Traits<S>::link>* __restrict__ Uq,
                                                  const int* __restrict__ nbrp,
                                                  const typename Traits<S>::kword* __restrict__ Ainv,
                                                  typename Traits<S>::word* __restrict__ y, int nrhs, int ntiles,
                                                  const int* __restrict__ order) {
    typedef typename Traits<S>::real R;
    const VItem it = vitem<RI, NT>(n2, nrhs, ntiles, order);
    const cx<typename Traits<S>::link>* Uf = Up;
    const typename Traits<S>::kword* Ak = Ainv;
    const int* nb = nbrp;
    unsigned kst = n2, l0 = 0, nstr = 0;
    if (STG) {
        const Staged<S> sd = stage_site_data<S, NT>(it, n2, nrhs, Up, Ainv, nbrp);
        Uf = sd.U;
        Ak = sd.K;
        nb = sd.nbr;
        kst = nstr = stg_sites<NT>();
        l0 = sd.l0;
    }
    if (!it.ok) return;
    const VView<RI, S> w(n2, nrhs, it.i, it.r);
    cx<R> acc[12], out[12];
    if (alpha != R(0))
        hop_sum<R, HOPS_ALL, hop_pipe<STG>(), site_major_links<S, RI>()>(n2, it.i, x + w.base, Uf, Uq, nb, acc, 8,
                                                              RI ? nrhs : 1, RI ? it.r : 0, w.stride, l0, nstr);
    else
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = mk(R(0), R(0));
    if (c) {
        cx<R> cc[12];
        load_spinor(c + w.base, w.stride, w.idx, cc);
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = cc[k] + alpha * acc[k];
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = alpha * acc[k];
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) out[k] = mk(R(0), R(0));
    apply_diag<R>(Ak, kst, it.i - l0, R(0), acc, out, R(0));
    store_spinor(y + w.base, w.stride, w.idx, out);
}

enum EoEpi { EOE_NONE = 0, EOE_DOT = 1, EOE_DOT4 = 2, EOE_RESID = 3 };

// y_p = [A_pp] c_p + beta H_{p,1-p} t (USE_A: clover + mass on c, else c itself).
// Epilogues as for the full operator: DOT partial (aux, y); DOT4 partials (y, c), (y, y),
// (aux, c), (aux, y); RESID: y = aux - y and partial ||y||^2.
template <class S, int EPI, bool USE_A, bool RI, bool STG, int NT>
__global__ __launch_bounds__(NT) void k_eo_diaghop(unsigned n2, const typename Traits<S>::word* __restrict__ c,
                                                   const typename Traits<S>::word* __restrict__ t,
                                                   typename Traits<S>::real beta,
                                                   const cx<typename Traits<S>::link>* __restrict__ Up,
                                                   const cx<typename Traits<S>::link>* __restrict__ Uq,
                                                   const int* __restrict__ nbrp,
                                                   const typename Traits<S>::kword* __restrict__ Kp,
                                                   typename Traits<S>::real mass4,
                                                   const typename Traits<S>::word* __restrict__ aux,
                                                   typename Traits<S>::word* __restrict__ y, double* part, int nrhs,
                                                   int ntiles, const int* __restrict__ order) {
    typedef typename Traits<S>::real R;
    const VItem it = vitem<RI, NT>(n2, nrhs, ntiles, order);
    const cx<typename Traits<S>::link>* Uf = Up;
    const typename Traits<S>::kword* Kk = Kp;
    const int* nb = nbrp;
    unsigned kst = n2, l0 = 0, nstr = 0;
    if (STG) {
        const Staged<S> sd = stage_site_data<S, NT>(it, n2, nrhs, Up, Kp, nbrp);
        Uf = sd.U;
        Kk = sd.K;
        nb = sd.nbr;
        kst = nstr = stg_sites<NT>();
        l0 = sd.l0;
    }
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    if (it.ok) {
        const VView<RI, S> w(n2, nrhs, it.i, it.r);
        cx<R> acc[12], cc[12];
        hop_sum<R, HOPS_ALL, hop_pipe<STG>(), site_major_links<S, RI>()>(n2, it.i, t + w.base, Uf, Uq, nb, acc, 8,
                                                              RI ? nrhs : 1, RI ? it.r : 0, w.stride, l0, nstr);
        load_spinor(c + w.base, w.stride, w.idx, cc);
        if (USE_A) {
            apply_diag<R>(Kk, kst, it.i - l0, mass4, cc, acc, beta);
        } else {
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[k] = cc[k] + beta * acc[k];
        }
        if (EPI == EOE_RESID) {
            cx<R> b[12];
            load_spinor(aux + w.base, w.stride, w.idx, b);
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[k] = b[k] - acc[k];
            v[0] = acc_nrm(acc);
        }
        store_spinor(y + w.base, w.stride, w.idx, acc);
        if (EPI == EOE_DOT) {
            cx<R> q[12];
            load_spinor(aux + w.base, w.stride, w.idx, q);
            acc_dot(q, acc, v[0], v[1]);
        }
        if (EPI == EOE_DOT4) {
            acc_dot(acc, cc, v[0], v[1]);
            v[2] = acc_nrm(acc);
            cx<R> q[12];
            load_spinor(aux + w.base, w.stride, w.idx, q);
            acc_dot(q, cc, v[3], v[4]);
            acc_dot(q, acc, v[5], v[6]);
        }
    }
    if (EPI == EOE_DOT) vpartials<2, RI, NT, R>(v, part, ntiles, it, nrhs);
    if (EPI == EOE_DOT4) vpartials<7, RI, NT, R>(v, part, ntiles, it, nrhs);
    if (EPI == EOE_RESID) vpartials<1, RI, NT, R>(v, part, ntiles, it, nrhs);
}

// Calls f(std::integral_constant<int, NT>) for the RHS-innermost workgroup size nt (FP64: WG only).
template <class S, class Fn>
static void with_op_threads(int nt, Fn&& f) {
    if constexpr (!std::is_same<S, double>::value) {
        switch (nt) {
            case 128: f(std::integral_constant<int, 128>()); return;
            case 512: f(std::integral_constant<int, 512>()); return;
            default: break;
        }
    }
    f(std::integral_constant<int, WG>());
}

template <class S>
void launch_eo_hopinv(Exec& e, const EoFields<S>& F, int p, bool ri, const typename Traits<S>::word* x,
                      const typename Traits<S>::word* c, double alpha, const typename Traits<S>::kword* Ainv,
                      typename Traits<S>::word* y, int nrhs, int kclass, double bytes) {
    typedef typename Traits<S>::real R;
    Timed t(e, kclass, bytes);
    const int nt = eo_op_tiles(F, nrhs, ri);
    if (!ri) {
        k_eo_hopinv<S, false, false, WG><<<nt * nrhs, WG, 0, e.stream>>>(F.n2, x, c, (R)alpha, F.U[p], F.U[1 - p],
                                                                         F.nbr[p], Ainv, y, nrhs, nt, nullptr);
        return;
    }
    const bool stg = stage_ok<S>(nrhs);
    with_op_threads<S>(eo_op_threads(F, nrhs, ri), [&](auto ntc) {
        constexpr int NT = decltype(ntc)::value;
        if (stg)
            k_eo_hopinv<S, true, true, NT><<<nt, NT, stage_bytes<S, NT>(), e.stream>>>(
                F.n2, x, c, (R)alpha, F.U[p], F.U[1 - p], F.nbr[p], Ainv, y, nrhs, nt, F.order);
        else
            k_eo_hopinv<S, true, false, NT><<<nt, NT, 0, e.stream>>>(F.n2, x, c, (R)alpha, F.U[p], F.U[1 - p],
                                                                     F.nbr[p], Ainv, y, nrhs, nt, F.order);
    });
}

template <class S>
void launch_eo_diaghop(Exec& e, const EoFields<S>& F, int p, bool ri, int epi, bool use_a,
                       const typename Traits<S>::word* c, const typename Traits<S>::word* tv, double beta,
                       double mass4, const typename Traits<S>::word* aux, typename Traits<S>::word* y, double* part,
                       int nrhs, int kclass, double bytes) {
    typedef typename Traits<S>::real R;
    Timed tm(e, kclass, bytes);
    const int nt = eo_op_tiles(F, nrhs, ri);
    const bool stg = ri && stage_ok<S>(nrhs);
    auto launch = [&](auto epc, auto uac, auto ric, auto ntc) {
        constexpr int EP = decltype(epc)::value, NT = decltype(ntc)::value;
        constexpr bool UA = decltype(uac)::value, RIV = decltype(ric)::value;
        const int ng = RIV ? nt : nt * nrhs;
        if (RIV && stg)
            k_eo_diaghop<S, EP, UA, RIV, RIV, NT><<<ng, NT, stage_bytes<S, NT>(), e.stream>>>(
                F.n2, c, tv, (R)beta, F.U[p], F.U[1 - p], F.nbr[p], F.K[p], (R)mass4, aux, y, part, nrhs, nt,
                RIV ? F.order : nullptr);
        else
            k_eo_diaghop<S, EP, UA, RIV, false, NT><<<ng, NT, 0, e.stream>>>(
                F.n2, c, tv, (R)beta, F.U[p], F.U[1 - p], F.nbr[p], F.K[p], (R)mass4, aux, y, part, nrhs, nt,
                RIV ? F.order : nullptr);
    };
    typedef std::integral_constant<bool, true> T_;
    typedef std::integral_constant<bool, false> F_;
    auto epilogue = [&](auto ric, auto ntc) {
        if (!use_a) {
            launch(std::integral_constant<int, EOE_NONE>(), F_(), ric, ntc);
            return;
        }
        switch (epi) {
            case EOE_DOT: launch(std::integral_constant<int, EOE_DOT>(), T_(), ric, ntc); break;
            case EOE_DOT4: launch(std::integral_constant<int, EOE_DOT4>(), T_(), ric, ntc); break;
            case EOE_RESID: launch(std::integral_constant<int, EOE_RESID>(), T_(), ric, ntc); break;
            default: launch(std::integral_constant<int, EOE_NONE>(), T_(), ric, ntc); break;
        }
    };
    if (ri)
        with_op_threads<S>(eo_op_threads(F, nrhs, ri), [&](auto ntc) { epilogue(T_(), ntc); });
    else
        epilogue(F_(), std::integral_constant<int, WG>());
}

#define EO_INST(S)                                                                                                 \
    template void launch_eo_hopinv<S>(Exec&, const EoFields<S>&, int, bool, const Traits<S>::word*,                \
                                      const Traits<S>::word*, double, const Traits<S>::kword*, Traits<S>::word*,   \
                                      int, int, double);                                                           \
    template void launch_eo_diaghop<S>(Exec&, const EoFields<S>&, int, bool, int, bool, const Traits<S>::word*,    \
                                       const Traits<S>::word*, double, double, const Traits<S>::word*,             \
                                       Traits<S>::word*, double*, int, int, double);
EO_INST(double)
EO_INST(float)
EO_INST(H16)

}  // namespace ddwc

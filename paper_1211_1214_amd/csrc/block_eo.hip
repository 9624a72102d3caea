// Even-odd preconditioned Schwarz block solves: x_k = D_k(m)^-1 b_k for every block k of
// one colour, with D_k the Dirichlet block operator (Sec. 1 of the paper).  Inside a
// block the odd sites are eliminated (eo.h):
//     M_k = A_ee - 1/4 H^k_eo A_oo^-1 H^k_oe,  b'_e = b_e + 1/2 H^k_eo A_oo^-1 b_o,
//     x_o = A_oo^-1 (b_o + 1/2 H^k_oe x_e),
// H^k the hops inside block k.  Every kernel here runs one workgroup per (block, RHS); the
// block's even and odd sites occupy the same contiguous range of the two half fields.
//   k_blk_prep    FP64: b'_e, r_e = b'_e, x_e = 0, ||b_k||^2, ||r_e||^2
//   k_blk_inner   persistent BiCGStab in precision R on M_k for r_e / ||r_e||, adds the
//                 correction to x_e in FP64 (blocks already converged return at once)
//   k_blk_resid   FP64: r_e = b'_e - M_k x_e and ||r_e||^2 (defect correction)
//   k_blk_recon   FP64: x_o, and (x_e, x_o) written to the full solution
#include <type_traits>

#include "ddwc_internal.h"
#include "eo.h"
#include "../../include/ddwc.h"

namespace ddwc {

constexpr int BE_MAX_THREADS = 256;  // FP64 kernels: prep, resid, recon and the FP64 inner solver
constexpr int BE_INNER_MAX = 768;    // FP32/FP16 inner solver: up to 12 waves (3 per SIMD at its VGPR use)

// Workgroup size of a block kernel of at most `cap` threads: `req` (a multiple of 64, from the
// schedule options) or, by default, enough waves for one block parity.
static int block_threads_for(const Geom& g, int req, int cap) {
    const int t = req > 0 ? ((req + 63) / 64) * 64 : ((g.hvb + 63) / 64) * 64;
    return t < cap ? t : cap;
}
int block_eo_threads(const Geom& g, int req) { return block_threads_for(g, req, BE_MAX_THREADS); }

// The persistent inner solver in FP32/FP16 storage runs up to BE_INNER_MAX threads: a 6^4 block
// parity (648 sites) is then one pass of 11 waves, and one such workgroup per CU keeps the
// block vectors in flight small enough for the last-level cache.
template <class S>
constexpr int be_inner_max() {
    return std::is_same<S, double>::value ? BE_MAX_THREADS : BE_INNER_MAX;
}

struct BlkIdx {
    int rank, rhs, B;
    unsigned h0;  // half index of the block's first site (both parities)
    size_t key;   // (rhs, rank) slot of the per-block arrays
};

// Workgroups are numbered block-major, RHS-minor and dealt to the 8 XCDs so that each XCD
// sweeps a contiguous range: the RHS of one block run on one XCD and share its links and
// clover in that XCD's L2.
__device__ __forceinline__ BlkIdx blk_idx(const Geom& g, int colour, int nrhs) {
    BlkIdx b;
    const int n = (int)gridDim.x;
    const int L = (n & 7) ? (int)blockIdx.x : ((int)blockIdx.x & 7) * (n >> 3) + ((int)blockIdx.x >> 3);
    b.rank = L / nrhs;
    b.rhs = L - b.rank * nrhs;
    b.B = colour * g.NBc + b.rank;
    b.h0 = (unsigned)b.B * g.hvb;
    b.key = (size_t)b.rhs * g.NBc + b.rank;
    return b;
}

// Ainv (c + alpha H^k x) at odd half site j (x even), into y (odd).
// Storage S (double, float or H16; arithmetic in Traits<S>::real).  A vector of one RHS is a
// slab of slab_words<S>(n2) words: the word planes and, for H16, the plane of site scales.
template <class S>
__host__ __device__ __forceinline__ size_t slab_words(unsigned n2) {
    return (size_t)Traits<S>::NCW * n2 + (std::is_same<S, H16>::value ? n2 / 4 : 0);
}

// Direction loop of the in-block hops (hop_sum): unrolled for FP64 and FP32 storage, rolled for
// FP16 (unrolled it spills).
template <class S>
constexpr int blk_hop_mode() {
    return std::is_same<S, H16>::value ? 0 : 2;
}

template <class S>
__device__ __forceinline__ void odd_pass(unsigned n2, unsigned j, const typename Traits<S>::word* x,
                                         const typename Traits<S>::word* c, typename Traits<S>::real alpha,
                                         const EoFields<S>& F, const typename Traits<S>::kword* Ainv,
                                         cx<typename Traits<S>::real> w[12]) {
    typedef typename Traits<S>::real R;
    cx<R> acc[12];
    hop_sum<R, HOPS_INSIDE, blk_hop_mode<S>()>(n2, j, x, F.U[1], F.U[0], F.nbr[1], acc, 8);
    if (c) {
        cx<R> cc[12];
        load_spinor(c, n2, j, cc);
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = cc[k] + alpha * acc[k];
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = alpha * acc[k];
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) w[k] = mk(R(0), R(0));
    apply_diag<R>(Ainv, n2, j, R(0), acc, w, R(0));
}

// [A_ee] c + beta H^k t at even half site i (t odd).
template <class S, bool USE_A>
__device__ __forceinline__ void even_pass(unsigned n2, unsigned i, const typename Traits<S>::word* c,
                                          const typename Traits<S>::word* t, typename Traits<S>::real beta,
                                          const EoFields<S>& F, typename Traits<S>::real mass4,
                                          cx<typename Traits<S>::real> y[12]) {
    typedef typename Traits<S>::real R;
    cx<R> cc[12];
    hop_sum<R, HOPS_INSIDE, blk_hop_mode<S>()>(n2, i, t, F.U[0], F.U[1], F.nbr[0], y, 8);
    load_spinor(c, n2, i, cc);
    if (USE_A) {
        apply_diag<R>(F.K[0], n2, i, mass4, cc, y, beta);
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) y[k] = cc[k] + beta * y[k];
    }
}

__global__ __launch_bounds__(BE_MAX_THREADS) void k_blk_prep(Geom g, EoFields<double> F, const double2* __restrict__ Ainv,
                                                            const double2* __restrict__ b, double2* __restrict__ bpe,
                                                            double2* __restrict__ re, double2* __restrict__ xe,
                                                            double2* __restrict__ to, double* bb, double* rr,
                                                            int colour, int nrhs) {
    __shared__ double lds[16];
    const BlkIdx k = blk_idx(g, colour, nrhs);
    const unsigned n2 = F.n2;
    const size_t of = (size_t)k.rhs * 12 * g.V, oh = (size_t)k.rhs * 12 * n2;
    double red[1] = {0};
    // odd pass: t_o = A_oo^-1 b_o ; ||b_o||^2
#pragma unroll 1
    for (int l = threadIdx.x; l < g.hvb; l += blockDim.x) {
        const unsigned j = k.h0 + l, s = full_index(g, j, 1);
        cx<double> bo[12], w[12], z[12];
        load_spinor(b + of, g.V, s, bo);
        red[0] += acc_nrm(bo);
#pragma unroll
        for (int c = 0; c < 12; ++c) w[c] = z[c] = mk(0.0, 0.0);
        apply_diag<double>(Ainv, n2, j, 0.0, bo, w, 0.0);
        store_spinor(to + oh, n2, j, w);
    }
    __syncthreads();
    // even pass: b'_e = b_e + 1/2 H^k t_o ; r_e = b'_e ; x_e = 0 ; ||b_e||^2, ||r_e||^2
    double red2[1] = {0};
#pragma unroll 1
    for (int l = threadIdx.x; l < g.hvb; l += blockDim.x) {
        const unsigned i = k.h0 + l, s = full_index(g, i, 0);
        cx<double> be[12], y[12], z[12];
        load_spinor(b + of, g.V, s, be);
        red[0] += acc_nrm(be);
        hop_sum<double, HOPS_INSIDE, 2>(n2, i, to + oh, F.U[0], F.U[1], F.nbr[0], y, 8);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            y[c] = be[c] + 0.5 * y[c];
            z[c] = mk(0.0, 0.0);
        }
        store_spinor(bpe + oh, n2, i, y);
        store_spinor(re + oh, n2, i, y);
        store_spinor(xe + oh, n2, i, z);
        red2[0] += acc_nrm(y);
    }
    block_sum<1>(red, lds);
    block_sum<1>(red2, lds);
    if (threadIdx.x == 0) {
        bb[k.key] = red[0];
        rr[k.key] = red2[0];
    }
}

__global__ __launch_bounds__(BE_MAX_THREADS) void k_blk_resid(Geom g, EoFields<double> F, const double2* __restrict__ Ainv,
                                                             const double2* __restrict__ bpe, const double2* __restrict__ xe,
                                                             double2* __restrict__ re, double2* __restrict__ to, double* rr,
                                                             double mass4, int colour, int nrhs) {
    __shared__ double lds[16];
    const BlkIdx k = blk_idx(g, colour, nrhs);
    const unsigned n2 = F.n2;
    const size_t oh = (size_t)k.rhs * 12 * n2;
#pragma unroll 1
    for (int l = threadIdx.x; l < g.hvb; l += blockDim.x) {
        cx<double> w[12];
        odd_pass<double>(n2, k.h0 + l, xe + oh, nullptr, 1.0, F, Ainv, w);
        store_spinor(to + oh, n2, k.h0 + l, w);
    }
    __syncthreads();
    double red[1] = {0};
#pragma unroll 1
    for (int l = threadIdx.x; l < g.hvb; l += blockDim.x) {
        const unsigned i = k.h0 + l;
        cx<double> y[12], bv[12];
        even_pass<double, true>(n2, i, xe + oh, to + oh, -0.25, F, mass4, y);
        load_spinor(bpe + oh, n2, i, bv);
#pragma unroll
        for (int c = 0; c < 12; ++c) y[c] = bv[c] - y[c];
        store_spinor(re + oh, n2, i, y);
        red[0] += acc_nrm(y);
    }
    block_sum<1>(red, lds);
    if (threadIdx.x == 0) rr[k.key] = red[0];
}

// x = (x_e, x_o) on the blocks of the colour with x_o = A_oo^-1 (b_o + 1/2 H^k x_e), assembled
// from the two parts the FP64 passes already hold: to = A_oo^-1 b_o (k_blk_prep) and, when a
// residual pass ran on the final x_e, th = A_oo^-1 H^k x_e (k_blk_resid; th null when x_e = 0).
__global__ __launch_bounds__(BE_MAX_THREADS) void k_blk_recon(Geom g, const double2* __restrict__ to,
                                                             const double2* __restrict__ th,
                                                             const double2* __restrict__ xe, double2* __restrict__ x,
                                                             int colour, int nrhs) {
    const BlkIdx k = blk_idx(g, colour, nrhs);
    const unsigned n2 = g.V / 2;
    const size_t of = (size_t)k.rhs * 12 * g.V, oh = (size_t)k.rhs * 12 * n2;
#pragma unroll 1
    for (int l = threadIdx.x; l < g.hvb; l += blockDim.x) {
        const unsigned j = k.h0 + l;
        cx<double> w[12], e[12];
        load_spinor(to + oh, n2, j, w);
        if (th) {
            cx<double> h[12];
            load_spinor(th + oh, n2, j, h);
#pragma unroll
            for (int c = 0; c < 12; ++c) w[c] = w[c] + 0.5 * h[c];
        }
        store_spinor(x + of, g.V, full_index(g, j, 1), w);
        load_spinor(xe + oh, n2, j, e);
        store_spinor(x + of, g.V, full_index(g, j, 0), e);
    }
    // the solution is zero on the other colour: clear the block of the other colour with the same
    // rank (sites (B2 * Vb .. B2 * Vb + Vb) of the full field), so every such block is cleared once
    const unsigned s0 = (unsigned)((1 - colour) * g.NBc + k.rank) * (unsigned)g.Vb;
    const cx<double> z[12] = {};
#pragma unroll 1
    for (int l = threadIdx.x; l < g.Vb; l += blockDim.x) store_spinor(x + of, g.V, s0 + l, z);
}

template <class S>
struct BlkInner {
    typedef typename Traits<S>::word W;
    typedef typename Traits<typename Traits<S>::xs>::word XW;
    W *r, *rh, *p, *v, *t, *tmp;
    XW* e;  // the correction, in Traits<S>::xs
};

template <class R>
__device__ __forceinline__ cx<R> cdiv_r(cx<double> a, cx<double> b) {
    const double d = b.re * b.re + b.im * b.im;
    return mk((R)((a.re * b.re + a.im * b.im) / d), (R)((a.im * b.re - a.re * b.im) / d));
}

// v = M_k p on the block (two passes separated by a workgroup barrier), with the dot
// products requested: (rh, v) when DOT1, (v, p) and (v, v) when DOT2.
template <class S, int DOT>
__device__ __forceinline__ void apply_Mk(const Geom& g, const EoFields<S>& F, const typename Traits<S>::kword* Ainv,
                                         unsigned h0, size_t oR, const typename Traits<S>::word* in,
                                         typename Traits<S>::word* tmp, typename Traits<S>::word* out,
                                         const typename Traits<S>::word* rh, typename Traits<S>::real mass4,
                                         double red[3]) {
    typedef typename Traits<S>::real R;
    const unsigned n2 = F.n2;
#pragma unroll 1
    for (int l = threadIdx.x; l < g.hvb; l += blockDim.x) {
        cx<R> w[12];
        odd_pass<S>(n2, h0 + l, in + oR, nullptr, R(1), F, Ainv, w);
        store_spinor(tmp + oR, n2, h0 + l, w);
    }
    __syncthreads();
#pragma unroll 1
    for (int l = threadIdx.x; l < g.hvb; l += blockDim.x) {
        const unsigned i = h0 + l;
        cx<R> y[12];
        even_pass<S, true>(n2, i, in + oR, tmp + oR, R(-0.25), F, mass4, y);
        store_spinor(out + oR, n2, i, y);
        if (DOT == 1) {
            cx<R> h[12];
            load_spinor(rh + oR, n2, i, h);
            acc_dot(h, y, red[0], red[1]);
        } else {
            cx<R> c[12];
            load_spinor(in + oR, n2, i, c);
            acc_dot(y, c, red[0], red[1]);
            red[2] += acc_nrm(y);
        }
    }
}

template <class S>
__global__ __launch_bounds__(be_inner_max<S>()) void k_blk_inner(Geom g, EoFields<S> F,
                                                             const typename Traits<S>::kword* __restrict__ Ainv,
                                                             const double2* __restrict__ re, double2* __restrict__ xe,
                                                             BlkInner<S> w, const double* __restrict__ bb,
                                                             const double* __restrict__ rr, double mass4, double tol,
                                                             double inner_floor, int maxit, int* iters, int colour,
                                                             int nrhs) {
    __shared__ double lds[3 * 16];
    const BlkIdx k = blk_idx(g, colour, nrhs);
    const double b2 = bb[k.key], r2 = rr[k.key];
    if (!(b2 > 0) || !(r2 > tol * tol * b2) || !isfinite(r2)) return;  // uniform over the workgroup
    const unsigned n2 = F.n2;
    typedef typename Traits<S>::real R;
    typedef typename Traits<S>::xs XS;
    const size_t oh = (size_t)k.rhs * 12 * n2, oR = (size_t)k.rhs * slab_words<S>(n2),
                 oX = (size_t)k.rhs * Traits<XS>::NCW * n2;
    const R m4 = (R)mass4;
    const double rn = sqrt(r2), sc = 1.0 / rn;
    double eps = 0.5 * tol * sqrt(b2) / rn;
    if (eps < inner_floor) eps = inner_floor;
    double red[3] = {0, 0, 0};
#pragma unroll 1
    for (int l = threadIdx.x; l < g.hvb; l += blockDim.x) {
        const unsigned i = k.h0 + l;
        cx<double> a[12];
        cx<R> q[12];
        cx<XS> z[12];
        load_spinor(re + oh, n2, i, a);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            q[c] = mk((R)(sc * a[c].re), (R)(sc * a[c].im));
            z[c] = mk(XS(0), XS(0));
        }
        store_spinor(w.r + oR, n2, i, q);
        store_spinor(w.rh + oR, n2, i, q);
        store_spinor(w.p + oR, n2, i, q);
        store_spinor(w.e + oX, n2, i, z);
        red[0] += acc_nrm(q);
    }
    block_sum<1>(red, lds);
    cx<double> rho = mk(red[0], 0.0);
    const double thr2 = eps * eps * red[0];
    int it = 0;
    while (it < maxit) {
        red[0] = red[1] = red[2] = 0;
        apply_Mk<S, 1>(g, F, Ainv, k.h0, oR, w.p, w.tmp, w.v, w.rh, m4, red);
        block_sum<2>(red, lds);
        if (!(red[0] * red[0] + red[1] * red[1] > 0)) break;
        const cx<R> alpha = cdiv_r<R>(rho, mk(red[0], red[1]));
        // s = r - alpha v (kept in r)
#pragma unroll 1
        for (int l = threadIdx.x; l < g.hvb; l += blockDim.x) {
            const unsigned i = k.h0 + l;
            cx<R> a[12], vv[12];
            load_spinor(w.r + oR, n2, i, a);
            load_spinor(w.v + oR, n2, i, vv);
#pragma unroll
            for (int c = 0; c < 12; ++c) a[c] = a[c] - alpha * vv[c];
            store_spinor(w.r + oR, n2, i, a);
        }
        __syncthreads();
        red[0] = red[1] = red[2] = 0;
        apply_Mk<S, 2>(g, F, Ainv, k.h0, oR, w.r, w.tmp, w.t, nullptr, m4, red);
        block_sum<3>(red, lds);
        cx<R> omega = mk(R(0), R(0));
        if (red[2] > 0) omega = mk((R)(red[0] / red[2]), (R)(red[1] / red[2]));
        // e += alpha p + omega s ; r = s - omega t ; (rh, r), (r, r)
        red[0] = red[1] = red[2] = 0;
#pragma unroll 1
        for (int l = threadIdx.x; l < g.hvb; l += blockDim.x) {
            const unsigned i = k.h0 + l;
            cx<XS> ee[12];
            cx<R> pp[12], ss[12], tt[12];
            load_spinor(w.e + oX, n2, i, ee);
            load_spinor(w.p + oR, n2, i, pp);
            load_spinor(w.r + oR, n2, i, ss);
            load_spinor(w.t + oR, n2, i, tt);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const cx<R> d = alpha * pp[c] + omega * ss[c];
                ee[c] = ee[c] + mk((XS)d.re, (XS)d.im);
                ss[c] = ss[c] - omega * tt[c];
            }
            store_spinor(w.e + oX, n2, i, ee);
            store_spinor(w.r + oR, n2, i, ss);
            load_spinor(w.rh + oR, n2, i, pp);
            acc_dot(pp, ss, red[0], red[1]);
            red[2] += acc_nrm(ss);
        }
        block_sum<3>(red, lds);
        ++it;
        if (red[2] <= thr2 || !isfinite(red[2])) break;
        if (omega.re == R(0) && omega.im == R(0)) break;
        const double d1 = rho.re * rho.re + rho.im * rho.im;
        if (!(d1 > 0)) break;
        const cx<double> q = mk((red[0] * rho.re + red[1] * rho.im) / d1, (red[1] * rho.re - red[0] * rho.im) / d1);
        const double d2 = (double)omega.re * omega.re + (double)omega.im * omega.im;
        const cx<double> ao = mk(((double)alpha.re * omega.re + (double)alpha.im * omega.im) / d2,
                                 ((double)alpha.im * omega.re - (double)alpha.re * omega.im) / d2);
        const cx<R> beta = mk((R)(q.re * ao.re - q.im * ao.im), (R)(q.re * ao.im + q.im * ao.re));
        rho = mk(red[0], red[1]);
#pragma unroll 1
        for (int l = threadIdx.x; l < g.hvb; l += blockDim.x) {
            const unsigned i = k.h0 + l;
            cx<R> a[12], pp[12], vv[12];
            load_spinor(w.r + oR, n2, i, a);
            load_spinor(w.p + oR, n2, i, pp);
            load_spinor(w.v + oR, n2, i, vv);
#pragma unroll
            for (int c = 0; c < 12; ++c) pp[c] = a[c] + beta * (pp[c] - omega * vv[c]);
            store_spinor(w.p + oR, n2, i, pp);
        }
        __syncthreads();
    }
    // x_e += ||r_e|| e in FP64
#pragma unroll 1
    for (int l = threadIdx.x; l < g.hvb; l += blockDim.x) {
        const unsigned i = k.h0 + l;
        cx<XS> e[12];
        cx<double> x[12];
        load_spinor(w.e + oX, n2, i, e);
        load_spinor(xe + oh, n2, i, x);
#pragma unroll
        for (int c = 0; c < 12; ++c) x[c] = x[c] + mk(rn * (double)e[c].re, rn * (double)e[c].im);
        store_spinor(xe + oh, n2, i, x);
    }
    if (threadIdx.x == 0) iters[k.key] += it;
}

// ------------------------------------------------------------------ LDS-resident inner solver
// The same BiCGStab on M_k as k_blk_inner, one workgroup per (block, RHS), for block parities of
// at most BL_MAX sites: one thread per local half index l < hvb owns the even site and the odd
// site of that index.  The operand of M_k (p, then s; even sites) and the odd intermediate
// A_oo^-1 H^k_oe (operand) are staged in LDS (2 x hvb x 96 bytes, 124 KB for a 6^4 block), so
// the in-block neighbour gathers of both passes, and each site's own operand, are LDS reads.
// r, p, v, rh and the correction e of a thread's own site are global slabs (slots 0, 2, 3, 1,
// 5), each read or written once or twice per iteration, so that no iterate stays live in
// registers across the stencil passes (s and t are formed in registers from the LDS operand and
// the even pass).  Links and clover are read from global
// memory: the RHS of one block run on one XCD and share them in its L2.  Arithmetic FP32, dot
// products accumulated in FP64 as in k_blk_inner.
constexpr int BL_MAX = 768;  // 12 waves: 3 per SIMD at up to 168 VGPRs

__device__ __forceinline__ void lds_load(const float4* __restrict__ L, unsigned HV, unsigned li, cx<float> q[12]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const float4 w = L[k * HV + li];
        q[2 * k] = mk(w.x, w.y);
        q[2 * k + 1] = mk(w.z, w.w);
    }
}
__device__ __forceinline__ void lds_store(float4* __restrict__ L, unsigned HV, unsigned li, const cx<float> q[12]) {
#pragma unroll
    for (int k = 0; k < 6; ++k)
        L[k * HV + li] = make_float4(q[2 * k].re, q[2 * k].im, q[2 * k + 1].re, q[2 * k + 1].im);
}

// acc = sum over the hops of half site s that stay inside its block (neighbour t with
// t - h0 < HV) of (1 -+ g_mu) W q(t), q read from LDS at t - h0; forward links Uf at s, backward
// links Ub at t (entry-major [4][9][n2]); nbr is the half-field table [8][n2] of s's parity.
// Software-pipelined: while hop d is applied, the link of hop d + 1 and the table entry of hop
// d + 2 are in flight (about one global latency per pass instead of one or two per hop).  The
// direction loop is unrolled: with a run-time direction the spin algebra sat behind a switch
// whose merge copied the accumulator and the prefetched link (42 moves per hop against 108
// arithmetic instructions); unrolled, the block kernel is 6.7% faster with identical results.
__device__ __forceinline__ void lds_hops(unsigned n2, unsigned s, unsigned h0, unsigned HV,
                                         const float4* __restrict__ L, const cx<float>* __restrict__ Uf,
                                         const cx<float>* __restrict__ Ub, const int* __restrict__ nbr,
                                         cx<float> acc[12]) {
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = mk(0.f, 0.f);
    int e = at(nbr, s), en = at(nbr + (size_t)n2, s);
    cx<float> u[9];
    {
        const unsigned t = e < 0 ? (unsigned)~e : (unsigned)e;
        if (t - h0 < HV) hop_link<LK_ENTRY>(Uf, Ub, n2, 0, s, t, u);
    }
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        const unsigned t = e < 0 ? (unsigned)~e : (unsigned)e;
        int enn = 0;
        if (d + 2 < 8) enn = at(nbr + (size_t)(d + 2) * n2, s);
        cx<float> un[9];
        if (d + 1 < 8) {
            const unsigned tn = en < 0 ? (unsigned)~en : (unsigned)en;
            if (tn - h0 < HV) hop_link<LK_ENTRY>(Uf, Ub, n2, d + 1, s, tn, un);
        }
        const unsigned li = t - h0;
        if (li < HV) {
            cx<float> q[12];
            lds_load(L, HV, li, q);
            if (e < 0) {
#pragma unroll
                for (int c = 0; c < 12; ++c) q[c] = -q[c];
            }
            hop_dispatch<float>(d, u, q, acc);
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) u[k] = un[k];
        e = en;
        en = enn;
    }
}

// w = A_oo^-1 H^k_oe q at odd half site j (q: even operand in LDS L).
__device__ __forceinline__ void odd_lds(const EoFields<float>& F, const float4* __restrict__ Ainv, unsigned j,
                                        unsigned h0, unsigned HV, const float4* __restrict__ L, cx<float> w[12]) {
    cx<float> acc[12];
    lds_hops(F.n2, j, h0, HV, L, F.U[1], F.U[0], F.nbr[1], acc);
#pragma unroll
    for (int c = 0; c < 12; ++c) w[c] = mk(0.f, 0.f);
    apply_diag<float>(Ainv, F.n2, j, 0.f, acc, w, 0.f);
}

// y = (4 + m + C) q_e - 1/4 H^k_eo q_o at even half site i: q_e the even operand in LDS Le (own
// site, local index l), q_o the odd intermediate in LDS Lo.
__device__ __forceinline__ void even_lds(const EoFields<float>& F, float m4, unsigned i, unsigned l, unsigned h0,
                                         unsigned HV, const float4* __restrict__ Le, const float4* __restrict__ Lo,
                                         cx<float> y[12]) {
    lds_hops(F.n2, i, h0, HV, Lo, F.U[0], F.U[1], F.nbr[0], y);
    cx<float> c[12];
    lds_load(Le, HV, l, c);
    apply_diag<float>(F.K[0], F.n2, i, m4, c, y, -0.25f);
}

__global__ __launch_bounds__(BL_MAX) void k_blk_lds(Geom g, EoFields<float> F, const float4* __restrict__ Ainv,
                                                    const double2* __restrict__ re, double2* __restrict__ xe,
                                                    float4* __restrict__ rg, float4* __restrict__ rhg, float4* __restrict__ pg,
                                                    float4* __restrict__ vg, float4* __restrict__ eg,
                                                    const double* __restrict__ bb, const double* __restrict__ rr,
                                                    double mass4, double tol, double inner_floor, int maxit,
                                                    int* iters, int colour, int nrhs) {
    extern __shared__ float4 bl_lds[];
    __shared__ double red_lds[2][8 * 16];  // alternating slots of the workgroup reductions
    const BlkIdx k = blk_idx(g, colour, nrhs);
    const double b2 = bb[k.key], r2 = rr[k.key];
    if (!(b2 > 0) || !(r2 > tol * tol * b2) || !isfinite(r2)) return;  // uniform over the workgroup
    const unsigned n2 = F.n2, HV = (unsigned)g.hvb, h0 = k.h0;
    float4* op = bl_lds;          // operand of M_k on the even sites of the block
    float4* tp = bl_lds + 6 * HV;  // A_oo^-1 H^k_oe (operand) on the odd sites
    const unsigned l = threadIdx.x;
    const bool act = l < HV;
    unsigned i = h0 + (act ? l : 0u);  // half index of this thread's even and odd site
    const size_t oh = (size_t)k.rhs * 12 * n2, oR = (size_t)k.rhs * 6 * n2;
    rg += oR;
    rhg += oR;
    pg += oR;
    vg += oR;
    eg += oR;
    const float m4 = (float)mass4;
    const double rn = sqrt(r2), sc = 1.0 / rn;
    double eps = 0.5 * tol * sqrt(b2) / rn;
    if (eps < inner_floor) eps = inner_floor;
    int phase = 0;  // reduction slot
    double red[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (act) {
        cx<double> a[12];
        load_spinor(re + oh, n2, i, a);
        cx<float> r[12], z[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            r[c] = mk((float)(sc * a[c].re), (float)(sc * a[c].im));
            z[c] = mk(0.f, 0.f);
        }
        store_spinor(rg, n2, i, r);
        store_spinor(rhg, n2, i, r);
        store_spinor(pg, n2, i, r);
        store_spinor(eg, n2, i, z);
        lds_store(op, HV, l, r);
        red[0] = acc_nrm(r);
    }
    block_sum1<1>(red, red_lds[phase ^= 1]);  // (its barrier also publishes the operand)
    cx<double> rho = mk(red[0], 0.0);
    const double thr2 = eps * eps * red[0];
    int it = 0;
    while (it < maxit) {
        // an opaque redefinition of the site index: keeps the compiler from hoisting every per-lane
        // 64-bit address out of the loop (they would not fit the 168 registers and would spill)
        asm volatile("" : "+v"(i));
        // v = M_k p, (rh, v)
        if (act) {
            cx<float> w[12];
            odd_lds(F, Ainv, i, h0, HV, op, w);
            lds_store(tp, HV, l, w);
        }
        __syncthreads();
        red[0] = red[1] = 0;
        if (act) {
            cx<float> v[12], h[12];
            even_lds(F, m4, i, l, h0, HV, op, tp, v);
            store_spinor(vg, n2, i, v);
            load_spinor(rhg, n2, i, h);
            acc_dot(h, v, red[0], red[1]);
        }
        block_sum1<2>(red, red_lds[phase ^= 1]);
        if (!(red[0] * red[0] + red[1] * red[1] > 0)) break;
        const cx<float> alpha = cdiv_r<float>(rho, mk(red[0], red[1]));
        // s = r - alpha v (kept in r), staged as the operand
        if (act) {
            cx<float> v[12], r[12];
            load_spinor(vg, n2, i, v);
            load_spinor(rg, n2, i, r);
#pragma unroll
            for (int c = 0; c < 12; ++c) r[c] = r[c] - alpha * v[c];
            lds_store(op, HV, l, r);
        }
        __syncthreads();
        // t = M_k s, (t, s), (t, t), (rh, s), (rh, t), (s, s)
        if (act) {
            cx<float> w[12];
            odd_lds(F, Ainv, i, h0, HV, op, w);
            lds_store(tp, HV, l, w);
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 8; ++c) red[c] = 0;
        cx<float> t[12];
        if (act) {
            even_lds(F, m4, i, l, h0, HV, op, tp, t);
            cx<float> sv[12], h[12];
            lds_load(op, HV, l, sv);
            acc_dot(t, sv, red[0], red[1]);
            red[2] = acc_nrm(t);
            load_spinor(rhg, n2, i, h);
            acc_dot(h, sv, red[3], red[4]);
            acc_dot(h, t, red[5], red[6]);
            red[7] = acc_nrm(sv);
        }
        block_sum1<8>(red, red_lds[phase ^= 1]);
        ++it;
        cx<float> omega = mk(0.f, 0.f);
        if (red[2] > 0) omega = mk((float)(red[0] / red[2]), (float)(red[1] / red[2]));
        // r = s - omega t is orthogonal to t, so ||r||^2 = (s, s) - |(t, s)|^2 / (t, t); the next
        // rho = (rh, r) = (rh, s) - omega (rh, t): one reduction serves omega, the stopping test and
        // beta, and x, r and p are updated in one pass
        const double r2n = red[2] > 0 ? red[7] - (red[0] * red[0] + red[1] * red[1]) / red[2] : red[7];
        const cx<double> rn_ = mk(red[3] - ((double)omega.re * red[5] - (double)omega.im * red[6]),
                                  red[4] - ((double)omega.re * red[6] + (double)omega.im * red[5]));
        const double d1 = rho.re * rho.re + rho.im * rho.im;
        const double d2 = (double)omega.re * omega.re + (double)omega.im * omega.im;
        const bool stop = r2n <= thr2 || !isfinite(r2n) || !(d2 > 0) || !(d1 > 0);
        cx<float> beta = mk(0.f, 0.f);
        if (!stop) {
            const cx<double> q = mk((rn_.re * rho.re + rn_.im * rho.im) / d1, (rn_.im * rho.re - rn_.re * rho.im) / d1);
            const cx<double> ao = mk(((double)alpha.re * omega.re + (double)alpha.im * omega.im) / d2,
                                     ((double)alpha.im * omega.re - (double)alpha.re * omega.im) / d2);
            beta = mk((float)(q.re * ao.re - q.im * ao.im), (float)(q.re * ao.im + q.im * ao.re));
        }
        rho = rn_;
        // e += alpha p + omega s ; r = s - omega t ; p = r + beta (p - omega v), staged as the next operand
        if (act) {
            cx<float> e[12], pp[12], r[12];
            lds_load(op, HV, l, r);
            load_spinor(eg, n2, i, e);
            load_spinor(pg, n2, i, pp);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                e[c] = e[c] + (alpha * pp[c] + omega * r[c]);
                r[c] = r[c] - omega * t[c];
            }
            store_spinor(eg, n2, i, e);
            if (!stop) {
                cx<float> v[12];
                store_spinor(rg, n2, i, r);
                load_spinor(vg, n2, i, v);
#pragma unroll
                for (int c = 0; c < 12; ++c) pp[c] = r[c] + beta * (pp[c] - omega * v[c]);
                store_spinor(pg, n2, i, pp);
                // (only this thread reads its own operand slot after the last barrier)
                lds_store(op, HV, l, pp);
            }
        }
        if (stop) break;
        __syncthreads();
    }
    // x_e += ||r_e|| e in FP64
    if (act) {
        cx<float> e[12];
        cx<double> x[12];
        load_spinor(eg, n2, i, e);
        load_spinor(xe + oh, n2, i, x);
#pragma unroll
        for (int c = 0; c < 12; ++c) x[c] = x[c] + mk(rn * (double)e[c].re, rn * (double)e[c].im);
        store_spinor(xe + oh, n2, i, x);
    }
    if (threadIdx.x == 0) iters[k.key] += it;
}

bool blk_lds_fits(const Geom& g, int lds_max_bytes) {
    return g.eo && g.hvb <= BL_MAX && (long long)2 * 6 * 16 * g.hvb + 3 * 16 * 8 <= lds_max_bytes;
}

void launch_blk_lds(Exec& e, const Geom& g, const EoFields<float>& F, const float4* Ainv, const double2* re,
                    double2* xe, void* const w[7], const double* bb, const double* rr, double mass4, double tol,
                    int maxit, int* iters, int colour, int nrhs) {
    Timed t(e, 2, 0);
    const int threads = ((g.hvb + 63) / 64) * 64;
    const size_t lds = (size_t)2 * 6 * g.hvb * sizeof(float4);
    // the inner solve stops at this relative residual at the least (FP32's reach)
    k_blk_lds<<<g.NBc * nrhs, threads, lds, e.stream>>>(g, F, Ainv, re, xe, (float4*)w[0], (float4*)w[1], (float4*)w[2],
                                                        (float4*)w[3], (float4*)w[5], bb, rr, mass4, tol, 2e-6,
                                                        maxit, iters, colour, nrhs);
}

void launch_blk_prep(Exec& e, const Geom& g, const EoFields<double>& F, const double2* Ainv, const double2* b,
                     double2* bpe, double2* re, double2* xe, double2* to, double* bb, double* rr, int colour, int nrhs) {
    Timed t(e, 4, 0);  // FP64 defect-correction passes: "other"
    k_blk_prep<<<g.NBc * nrhs, block_eo_threads(g, e.blk_threads), 0, e.stream>>>(g, F, Ainv, b, bpe, re, xe, to, bb, rr, colour, nrhs);
}
void launch_blk_resid(Exec& e, const Geom& g, const EoFields<double>& F, const double2* Ainv, const double2* bpe,
                      const double2* xe, double2* re, double2* to, double* rr, double mass4, int colour, int nrhs) {
    Timed t(e, 4, 0);  // FP64 defect-correction passes: "other"
    k_blk_resid<<<g.NBc * nrhs, block_eo_threads(g, e.blk_threads), 0, e.stream>>>(g, F, Ainv, bpe, xe, re, to, rr, mass4, colour,
                                                                    nrhs);
}
void launch_blk_recon(Exec& e, const Geom& g, const double2* to, const double2* th, const double2* xe, double2* x,
                      int colour, int nrhs) {
    Timed t(e, 4, 0);  // FP64 defect-correction passes: "other"
    k_blk_recon<<<g.NBc * nrhs, block_eo_threads(g, e.blk_threads), 0, e.stream>>>(g, to, th, xe, x, colour, nrhs);
}
template <class S>
void launch_blk_inner(Exec& e, const Geom& g, const EoFields<S>& F, const typename Traits<S>::kword* Ainv,
                      const double2* re, double2* xe, void* const w[7], const double* bb, const double* rr,
                      double mass4, double tol, int maxit, int* iters, int colour, int nrhs) {
    Timed t(e, 2, 0);
    BlkInner<S> bw;
    typedef typename Traits<S>::word W;
    bw.r = (W*)w[0];
    bw.rh = (W*)w[1];
    bw.p = (W*)w[2];
    bw.v = (W*)w[3];
    bw.t = (W*)w[4];
    bw.e = (typename BlkInner<S>::XW*)w[5];
    bw.tmp = (W*)w[6];
    // the inner solve stops at this relative residual at the least (the storage's reach)
    const double floor_eps = std::is_same<S, double>::value ? 0.0 : std::is_same<S, H16>::value ? 1e-3 : 2e-6;
    // e.blk_lds KiB of dynamic LDS (unused by the kernel) caps the workgroups resident per CU, and so
    // the slabs in flight, which then stay in the last-level cache
    k_blk_inner<S><<<g.NBc * nrhs, block_threads_for(g, e.blk_threads, be_inner_max<S>()), (size_t)e.blk_lds << 10,
                     e.stream>>>(g, F, Ainv, re, xe, bw, bb, rr, mass4, tol,
                                                                       floor_eps, maxit, iters, colour, nrhs);
}
size_t blk_slab_bytes(int prec, unsigned n2) {
    if (prec == DDWC_FP64) return slab_words<double>(n2) * 16;
    if (prec == DDWC_MIXED16) return slab_words<H16>(n2) * 16;
    return slab_words<float>(n2) * 16;
}
template void launch_blk_inner<double>(Exec&, const Geom&, const EoFields<double>&, const double2*, const double2*,
                                       double2*, void* const[7], const double*, const double*, double, double, int,
                                       int*, int, int);
template void launch_blk_inner<float>(Exec&, const Geom&, const EoFields<float>&, const float4*, const double2*,
                                      double2*, void* const[7], const double*, const double*, double, double, int,
                                      int*, int, int);
template void launch_blk_inner<H16>(Exec&, const Geom&, const EoFields<H16>&, const float4*, const double2*,
                                    double2*, void* const[7], const double*, const double*, double, double, int,
                                    int*, int, int);

}  // namespace ddwc

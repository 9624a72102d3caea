// Persistent Schwarz block solver: x_k = D_k(m)^-1 b_k for every block k of one colour
// (the Dirichlet block operators on the diagonal of D_bb or D_ww, Sec. 1 of the paper).
//
// One workgroup owns one (block, RHS) pair for the whole solve.  Block-major site order
// makes the block's sites contiguous, so every vector access is unit-stride inside the
// block; the Dirichlet operator only ever reads sites of the same block, so a workgroup
// barrier is the only synchronisation the Krylov iteration needs.  Dot products are
// workgroup reductions (wave shuffles + LDS, fixed order).  Blocks converge and exit
// independently.
//
// Inner precision R: BiCGStab on the scaled residual; outer loop in FP64: the true
// residual b - D_k x is recomputed with FP64 links and clover after every inner solve
// and the correction is accumulated in FP64 (defect correction).
#include "ddwc_internal.h"

namespace ddwc {

constexpr int BS_MAX_THREADS = 256;

int block_solver_threads(const Geom& g) {
    int t = ((g.Vb + 63) / 64) * 64;
    return t < BS_MAX_THREADS ? t : BS_MAX_THREADS;
}

template <class R>
struct Inner {
    typedef typename Traits<R>::word W;
    W *r, *rh, *p, *v, *t, *e;
};

template <class R>
__device__ __forceinline__ void ldv(const typename Traits<R>::word* f, size_t off, int V, int s, cx<R> a[12]) {
    load_spinor(f + off, V, s, a);
}
template <class R>
__device__ __forceinline__ void stv(typename Traits<R>::word* f, size_t off, int V, int s, const cx<R> a[12]) {
    store_spinor(f + off, V, s, a);
}

template <class R>
__device__ __forceinline__ cx<R> cdiv(cx<double> a, cx<double> b) {
    double d = b.re * b.re + b.im * b.im;
    return mk((R)((a.re * b.re + a.im * b.im) / d), (R)((a.im * b.re - a.re * b.im) / d));
}

template <class R>
__global__ __launch_bounds__(BS_MAX_THREADS) void k_block_solve(
    Geom g, const cx<double>* __restrict__ U64, const double2* __restrict__ K64, const cx<R>* __restrict__ UR,
    const typename Traits<R>::word* __restrict__ KR, const double2* __restrict__ b, double2* __restrict__ x,
    double2* __restrict__ r64, Inner<R> w, int colour, int nrhs, double mass4, double tol, int maxit,
    double inner_floor, int* iters, int* outer, double* relres, const int* __restrict__ nbr, int ndir) {
    typedef typename Traits<R>::word W;
    __shared__ double lds[4 * 16];
    const int rank = blockIdx.x / nrhs;
    const int rhs = blockIdx.x - rank * nrhs;
    const int base = (colour * g.NBc + rank) * g.Vb;
    const int V = g.V;
    const size_t o64 = (size_t)rhs * 12 * V;
    const size_t oR = (size_t)rhs * Traits<R>::NCW * V;
    const R m4 = (R)mass4;

    // ||b||^2, x = 0, r64 = b
    double red[4];
    red[0] = 0;
#pragma unroll 1
    for (int l = threadIdx.x; l < g.Vb; l += blockDim.x) {
        const int s = base + l;
        cx<double> a[12], z[12];
        load_spinor(b + o64, V, s, a);
        store_spinor(r64 + o64, V, s, a);
        for (int k = 0; k < 12; ++k) z[k] = mk(0.0, 0.0);
        store_spinor(x + o64, V, s, z);
        red[0] += acc_nrm(a);
    }
    block_sum<1>(red, lds);
    const double bb = red[0];
    double rr = bb;
    int total = 0, nout = 0;
    const double tol2bb = tol * tol * bb;

    while (bb > 0 && rr > tol2bb && total < maxit && isfinite(rr)) {
        ++nout;
        const double rn = sqrt(rr);
        const double sc = 1.0 / rn;
        double eps = 0.5 * tol * sqrt(bb) / rn;
        if (eps < inner_floor) eps = inner_floor;
        // r = rh = p = sc * r64, e = 0, rho = ||r||^2
        red[0] = 0;
#pragma unroll 1
    for (int l = threadIdx.x; l < g.Vb; l += blockDim.x) {
            const int s = base + l;
            cx<double> a[12];
            cx<R> q[12], z[12];
            load_spinor(r64 + o64, V, s, a);
            for (int k = 0; k < 12; ++k) {
                q[k] = mk((R)(sc * a[k].re), (R)(sc * a[k].im));
                z[k] = mk(R(0), R(0));
            }
            stv<R>(w.r, oR, V, s, q);
            stv<R>(w.rh, oR, V, s, q);
            stv<R>(w.p, oR, V, s, q);
            stv<R>(w.e, oR, V, s, z);
            red[0] += acc_nrm(q);
        }
        block_sum<1>(red, lds);  // also orders the stores above before the first operator
        cx<double> rho = mk(red[0], 0.0);
        const double thr2 = eps * eps * red[0];
        while (total < maxit) {
            // v = D_k p ; (rh, v)
            red[0] = red[1] = 0;
    #pragma unroll 1
    for (int l = threadIdx.x; l < g.Vb; l += blockDim.x) {
                const int s = base + l;
                cx<R> y[12], h[12];
                site_operator<R, true, HOPS_INSIDE>(g, s, w.p + oR, UR, KR, nbr, m4, y, ndir);
                stv<R>(w.v, oR, V, s, y);
                ldv<R>(w.rh, oR, V, s, h);
                acc_dot(h, y, red[0], red[1]);
            }
            block_sum<2>(red, lds);
            if (!(red[0] * red[0] + red[1] * red[1] > 0)) break;
            const cx<R> alpha = cdiv<R>(rho, mk(red[0], red[1]));
            // s = r - alpha v (kept in r)
    #pragma unroll 1
    for (int l = threadIdx.x; l < g.Vb; l += blockDim.x) {
                const int s = base + l;
                cx<R> rr_[12], vv[12];
                ldv<R>(w.r, oR, V, s, rr_);
                ldv<R>(w.v, oR, V, s, vv);
                for (int k = 0; k < 12; ++k) rr_[k] = rr_[k] - alpha * vv[k];
                stv<R>(w.r, oR, V, s, rr_);
            }
            __syncthreads();
            // t = D_k s ; (t, s), (t, t)
            red[0] = red[1] = red[2] = 0;
    #pragma unroll 1
    for (int l = threadIdx.x; l < g.Vb; l += blockDim.x) {
                const int s = base + l;
                cx<R> y[12], c[12];
                site_operator<R, true, HOPS_INSIDE>(g, s, w.r + oR, UR, KR, nbr, m4, y, ndir);
                stv<R>(w.t, oR, V, s, y);
                ldv<R>(w.r, oR, V, s, c);
                acc_dot(y, c, red[0], red[1]);
                red[2] += acc_nrm(y);
            }
            block_sum<3>(red, lds);
            cx<R> omega = mk(R(0), R(0));
            if (red[2] > 0) omega = mk((R)(red[0] / red[2]), (R)(red[1] / red[2]));
            // e += alpha p + omega s ; r = s - omega t ; (rh, r), (r, r)
            red[0] = red[1] = red[2] = 0;
    #pragma unroll 1
    for (int l = threadIdx.x; l < g.Vb; l += blockDim.x) {
                const int s = base + l;
                cx<R> ee[12], pp[12], ss[12], tt[12];
                ldv<R>(w.e, oR, V, s, ee);
                ldv<R>(w.p, oR, V, s, pp);
                ldv<R>(w.r, oR, V, s, ss);
                ldv<R>(w.t, oR, V, s, tt);
                for (int k = 0; k < 12; ++k) {
                    ee[k] = ee[k] + alpha * pp[k] + omega * ss[k];
                    ss[k] = ss[k] - omega * tt[k];
                }
                stv<R>(w.e, oR, V, s, ee);
                stv<R>(w.r, oR, V, s, ss);
                ldv<R>(w.rh, oR, V, s, pp);
                acc_dot(pp, ss, red[0], red[1]);
                red[2] += acc_nrm(ss);
            }
            block_sum<3>(red, lds);
            ++total;
            if (red[2] <= thr2 || !isfinite(red[2])) break;
            if (omega.re == R(0) && omega.im == R(0)) break;
            // beta = (rho_new / rho) (alpha / omega)
            const cx<double> rn_ = mk(red[0], red[1]);
            double d1 = rho.re * rho.re + rho.im * rho.im;
            if (!(d1 > 0)) break;
            cx<double> q = mk((rn_.re * rho.re + rn_.im * rho.im) / d1, (rn_.im * rho.re - rn_.re * rho.im) / d1);
            double d2 = (double)omega.re * omega.re + (double)omega.im * omega.im;
            cx<double> ao = mk(((double)alpha.re * omega.re + (double)alpha.im * omega.im) / d2,
                               ((double)alpha.im * omega.re - (double)alpha.re * omega.im) / d2);
            const cx<R> beta = mk((R)(q.re * ao.re - q.im * ao.im), (R)(q.re * ao.im + q.im * ao.re));
            rho = rn_;
            // p = r + beta (p - omega v)
    #pragma unroll 1
    for (int l = threadIdx.x; l < g.Vb; l += blockDim.x) {
                const int s = base + l;
                cx<R> rr_[12], pp[12], vv[12];
                ldv<R>(w.r, oR, V, s, rr_);
                ldv<R>(w.p, oR, V, s, pp);
                ldv<R>(w.v, oR, V, s, vv);
                for (int k = 0; k < 12; ++k) pp[k] = rr_[k] + beta * (pp[k] - omega * vv[k]);
                stv<R>(w.p, oR, V, s, pp);
            }
            __syncthreads();
        }
        // x += e / sc in FP64
#pragma unroll 1
    for (int l = threadIdx.x; l < g.Vb; l += blockDim.x) {
            const int s = base + l;
            cx<R> ee[12];
            cx<double> xx[12];
            ldv<R>(w.e, oR, V, s, ee);
            load_spinor(x + o64, V, s, xx);
            for (int k = 0; k < 12; ++k) xx[k] = xx[k] + mk(rn * (double)ee[k].re, rn * (double)ee[k].im);
            store_spinor(x + o64, V, s, xx);
        }
        __syncthreads();
        // r64 = b - D_k x in FP64
        red[0] = 0;
#pragma unroll 1
    for (int l = threadIdx.x; l < g.Vb; l += blockDim.x) {
            const int s = base + l;
            cx<double> y[12], bv[12];
            site_operator<double, true, HOPS_INSIDE>(g, s, x + o64, U64, K64, nbr, mass4, y, ndir);
            load_spinor(b + o64, V, s, bv);
            for (int k = 0; k < 12; ++k) y[k] = bv[k] - y[k];
            store_spinor(r64 + o64, V, s, y);
            red[0] += acc_nrm(y);
        }
        block_sum<1>(red, lds);
        rr = red[0];
        if (nout >= 64) break;
    }
    if (threadIdx.x == 0) {
        const int k = rhs * g.NBc + rank;
        iters[k] = total;
        outer[k] = nout;
        relres[k] = bb > 0 ? sqrt(rr / bb) : 0.0;
    }
}

void launch_block_solve64(Exec& e, const Geom& g, const cx<double>* U, const double2* K, const BlockSolveArgs& a) {
    Timed t(e, 2, 0);
    Inner<double> w;
    w.r = (double2*)a.w[0];
    w.rh = (double2*)a.w[1];
    w.p = (double2*)a.w[2];
    w.v = (double2*)a.w[3];
    w.t = (double2*)a.w[4];
    w.e = (double2*)a.w[5];
    k_block_solve<double><<<g.NBc * a.nrhs, block_solver_threads(g), 0, e.stream>>>(
        g, U, K, U, K, a.b, a.x, a.r64, w, a.colour, a.nrhs, a.mass4, a.tol, a.maxit, 0.0, a.iters, a.outer,
        a.relres, e.nbr, 8);
}

void launch_block_solve32(Exec& e, const Geom& g, const cx<double>* U64, const double2* K64, const cx<float>* U32,
                          const float4* K32, const BlockSolveArgs& a) {
    Timed t(e, 2, 0);
    Inner<float> w;
    w.r = (float4*)a.w[0];
    w.rh = (float4*)a.w[1];
    w.p = (float4*)a.w[2];
    w.v = (float4*)a.w[3];
    w.t = (float4*)a.w[4];
    w.e = (float4*)a.w[5];
    k_block_solve<float><<<g.NBc * a.nrhs, block_solver_threads(g), 0, e.stream>>>(
        g, U64, K64, U32, K32, a.b, a.x, a.r64, w, a.colour, a.nrhs, a.mass4, a.tol, a.maxit, 2e-6, a.iters,
        a.outer, a.relres, e.nbr, 8);
}

}  // namespace ddwc

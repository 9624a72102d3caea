// Derivatives of the exponents with respect to the links: the force kernels.
//
// Every link derivative of the estimator reduces to terms Re <a, (dD/dU) b> for pairs of
// full-lattice FP64 fields (a, b) with one weight per RHS.  The gradient is returned in the
// convention G = dL/dRe U + i dL/dIm U for each 3x3 link matrix U (no unitarity
// constraint); for a term Re tr[U Z] it is Z^+.
//
// Hops (D = (4 + m) + C - H/2):  the link U = U_mu(x) enters
//     a(x)^+ (1 - g_mu) U b(x + mu) + a(x + mu)^+ (1 + g_mu) U^+ b(x),
// times the time-boundary sign, so that G += -1/2 s [sum_alpha a_alpha(x) ((1 - g_mu) b(x + mu))_alpha^+
//                                                 + b_alpha(x) ((1 + g_mu) a(x + mu))_alpha^+]
// (colour outer products, spin summed).
//
// Clover (chiral blocks C_k = (i c_sw / 2) sum_l s_l x E_l^k, E from the field strengths as in
// clover_build.h):  Re <a, C b> = sum_x sum_{mu<nu} Re tr[Fhat_mu nu K_mu nu] with
// K = (i c_sw / 2) (signed sums of L_l^k), (L_l^k)_{ba} = sum_{alpha beta in block k} (s_l)_{alpha beta}
// b_{beta b} conj(a_{alpha a}); with Fhat = (Q - Q^+)/8 this is Re tr[Q J], J = (K - K^+)/8, and the
// link at position p of a leaf A X B contributes (B J A)^+ (X = U) or B J A (X = U^+).
#include "ddwc_internal.h"
#include "force.h"

namespace ddwc {

// in-place gamma_5 = diag(1, 1, -1, -1) on the spin index (chiral basis)
__global__ void k_gamma5(Geom g, double2* __restrict__ v, int nrhs) {
    const unsigned s = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= (unsigned)g.V) return;
    double2* f = v + (size_t)r * 12 * g.V;
#pragma unroll
    for (int c = 6; c < 12; ++c) {
        double2 w = f[(size_t)c * g.V + s];
        f[(size_t)c * g.V + s] = make_double2(-w.x, -w.y);
    }
}

void launch_gamma5(Exec& e, const Geom& g, double2* v, int nrhs) {
    Timed t(e, 4, 0);
    k_gamma5<<<dim3(tiles_of(g.V), nrhs), WG, 0, e.stream>>>(g, v, nrhs);
}

// G_mu(x) += hop part, one thread per (x, mu).
__global__ void k_force_hop(Geom g, const int* __restrict__ nbr, const double2* __restrict__ a,
                            const double2* __restrict__ b, const double* __restrict__ w, int nrhs,
                            cx<double>* __restrict__ G) {
    const unsigned s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= (unsigned)g.V) return;
    force_hop_site(g, nbr, a, b, w, nrhs, G, s, blockIdx.y);
}

void launch_force_hop(Exec& e, const Geom& g, const int* nbr, const double2* a, const double2* b, const double* w,
                      int nrhs, cx<double>* G) {
    Timed t(e, 4, 0);
    k_force_hop<<<dim3(tiles_of(g.V), 4), WG, 0, e.stream>>>(g, nbr, a, b, w, nrhs, G);
}

struct AtomicAdder {
    cx<double>* G;
    unsigned V;
    __device__ void operator()(int mu, int s, const M3& m) const {
        for (int k = 0; k < 9; ++k) {
            double* p = (double*)&G[((size_t)mu * 9 + k) * V + s];
            atomicAdd(p, m.a[k].re);
            atomicAdd(p + 1, m.a[k].im);
        }
    }
};

// One thread per site y: the clover part, scattered to the links of the leaves with atomic adds.
__global__ __launch_bounds__(128) void k_force_clover(Geom g, const cx<double>* __restrict__ U, double csw,
                                                      const double2* __restrict__ a, const double2* __restrict__ b,
                                                      const double* __restrict__ w, int nrhs,
                                                      cx<double>* __restrict__ G) {
    const int y = blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= g.V) return;
    force_clover_site(g, U, csw, a, b, w, nrhs, y, AtomicAdder{G, (unsigned)g.V});
}

void launch_force_clover(Exec& e, const Geom& g, const cx<double>* U, double csw, const double2* a, const double2* b,
                         const double* w, int nrhs, cx<double>* G) {
    Timed t(e, 4, 0);
    k_force_clover<<<(g.V + 127) / 128, 128, 0, e.stream>>>(g, U, csw, a, b, w, nrhs, G);
}

// internal [4][9][V] -> canonical [4][V][3][3]
__global__ void k_links_export(Geom g, const cx<double>* __restrict__ G, double2* __restrict__ can) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int mu = blockIdx.y;
    if (s >= g.V) return;
    const Site S = decode(g, s);
    double2* dst = can + ((size_t)mu * g.V + canonical_index(g, S)) * 9;
    for (int k = 0; k < 9; ++k) {
        const cx<double> v = G[((size_t)mu * 9 + k) * g.V + s];
        dst[k] = make_double2(v.re, v.im);
    }
}

void launch_links_export(Exec& e, const Geom& g, const cx<double>* G, void* canon) {
    Timed t(e, 4, 0);
    k_links_export<<<dim3(tiles_of(g.V), 4), WG, 0, e.stream>>>(g, G, (double2*)canon);
}

}  // namespace ddwc

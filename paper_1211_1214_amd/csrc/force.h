// Per-site logic of the link-derivative (force) kernels, shared with host-side checks.
// The formulas are stated in grad.hip.
#pragma once
#include "clover_build.h"

namespace ddwc {

// (1 + sgn g_mu) q on the 4 x 3 spinor q[spin * 3 + colour], MU fixed at compile time:
//   g_0 q = (-q_l, -q_u),  g_k q = (-i s_k q_l, i s_k q_u)  (u = spins 0,1; l = spins 2,3).
template <int MU>
DDWC_HD void proj(double sgn, const cx<double> q[12], cx<double> o[12]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cx<double> u0 = q[a], u1 = q[3 + a], l0 = q[6 + a], l1 = q[9 + a];
        cx<double> g0, g1, g2, g3;  // gamma_mu q, spins 0..3
        if (MU == 0) {
            g0 = -l0; g1 = -l1; g2 = -u0; g3 = -u1;
        } else if (MU == 1) {  // s_1 = [[0,1],[1,0]]
            g0 = times_mi(l1); g1 = times_mi(l0); g2 = times_i(u1); g3 = times_i(u0);
        } else if (MU == 2) {  // s_2 = [[0,-i],[i,0]]:  -i s_2 (l0,l1) = (-l1, l0), i s_2 (u0,u1) = (u1, -u0)
            g0 = -l1; g1 = l0; g2 = u1; g3 = -u0;
        } else {  // s_3 = diag(1,-1)
            g0 = times_mi(l0); g1 = times_i(l1); g2 = times_i(u0); g3 = times_mi(u1);
        }
        o[a] = u0 + sgn * g0;
        o[3 + a] = u1 + sgn * g1;
        o[6 + a] = l0 + sgn * g2;
        o[9 + a] = l1 + sgn * g3;
    }
}

DDWC_HD void ld12(const double2* f, unsigned V, unsigned s, cx<double> p[12]) {
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const double2 w = f[(size_t)c * V + s];
        p[c] = mk(w.x, w.y);
    }
}

// Hop part of the gradient of sum_r w_r Re <a_r, D b_r> at link (x = s, MU), added to G.
template <int MU>
DDWC_HD void force_hop_site_t(const Geom& g, const int* nbr, const double2* a, const double2* b, const double* w,
                              int nrhs, cx<double>* G, unsigned s) {
    const int e = nbr[(size_t)(2 * MU) * g.V + s];
    const unsigned t = e < 0 ? (unsigned)~e : (unsigned)e;
    const double sg = e < 0 ? -1.0 : 1.0;
    cx<double> acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = mk(0.0, 0.0);
    for (int r = 0; r < nrhs; ++r) {
        const double wr = w[r];
        if (wr == 0.0) continue;
        const double2* ar = a + (size_t)r * 12 * g.V;
        const double2* br = b + (size_t)r * 12 * g.V;
        cx<double> as[12], bs[12], pb[12], pa[12];
        {
            cx<double> q[12];
            ld12(br, g.V, t, q);
            proj<MU>(-1.0, q, pb);  // (1 - g_mu) b(x + mu)
            ld12(ar, g.V, t, q);
            proj<MU>(+1.0, q, pa);  // (1 + g_mu) a(x + mu)
        }
        ld12(ar, g.V, s, as);
        ld12(br, g.V, s, bs);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                cx<double> z = mk(0.0, 0.0);
#pragma unroll
                for (int al = 0; al < 4; ++al) {
                    z = z + as[3 * al + i] * mk(pb[3 * al + j].re, -pb[3 * al + j].im);
                    z = z + bs[3 * al + i] * mk(pa[3 * al + j].re, -pa[3 * al + j].im);
                }
                acc[3 * i + j] = acc[3 * i + j] + (-0.5 * sg * wr) * z;
            }
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        cx<double>& o = G[((size_t)MU * 9 + k) * g.V + s];
        o = o + acc[k];
    }
}

DDWC_HD void force_hop_site(const Geom& g, const int* nbr, const double2* a, const double2* b, const double* w,
                            int nrhs, cx<double>* G, unsigned s, int mu) {
    switch (mu) {
        case 0: force_hop_site_t<0>(g, nbr, a, b, w, nrhs, G, s); break;
        case 1: force_hop_site_t<1>(g, nbr, a, b, w, nrhs, G, s); break;
        case 2: force_hop_site_t<2>(g, nbr, a, b, w, nrhs, G, s); break;
        default: force_hop_site_t<3>(g, nbr, a, b, w, nrhs, G, s); break;
    }
}

// Clover part of the gradient of sum_r w_r Re <a_r, D b_r> from the clover term at site y:
// add(dir, site, Z) receives the contribution Z to the gradient of link (site, dir).
template <class ADD>
DDWC_HD void force_clover_site(const Geom& g, const cx<double>* U, double csw, const double2* a, const double2* b,
                               const double* w, int nrhs, int y, const ADD& add) {
    // L[k][l]: chiral block k, Pauli matrix l + 1
    M3 L[2][3];
    for (int k = 0; k < 2; ++k)
        for (int l = 0; l < 3; ++l)
            for (int q = 0; q < 9; ++q) L[k][l].a[q] = mk(0.0, 0.0);
    for (int r = 0; r < nrhs; ++r) {
        const double wr = w[r];
        if (wr == 0.0) continue;
        cx<double> av[12], bv[12];
        ld12(a + (size_t)r * 12 * g.V, g.V, y, av);
        ld12(b + (size_t)r * 12 * g.V, g.V, y, bv);
        for (int k = 0; k < 2; ++k) {
            const cx<double>* a0 = av + 6 * k;  // spin 2k, colours 0..2
            const cx<double>* a1 = av + 6 * k + 3;
            const cx<double>* b0 = bv + 6 * k;
            const cx<double>* b1 = bv + 6 * k + 3;
            for (int bb = 0; bb < 3; ++bb)
                for (int aa = 0; aa < 3; ++aa) {
                    // (L_l)_{bb aa} = sum_{al be} (s_l)_{al be} b_{be bb} conj(a_{al aa})
                    const cx<double> ca0 = mk(a0[aa].re, -a0[aa].im), ca1 = mk(a1[aa].re, -a1[aa].im);
                    const cx<double> t01 = b1[bb] * ca0;  // (al, be) = (0, 1)
                    const cx<double> t10 = b0[bb] * ca1;  // (1, 0)
                    const cx<double> t00 = b0[bb] * ca0;
                    const cx<double> t11 = b1[bb] * ca1;
                    const int q = 3 * bb + aa;
                    L[k][0].a[q] = L[k][0].a[q] + wr * (t01 + t10);
                    L[k][1].a[q] = L[k][1].a[q] + wr * (times_mi(t01) + times_i(t10));
                    L[k][2].a[q] = L[k][2].a[q] + wr * (t00 - t11);
                }
        }
    }
    // planes (0,1) (0,2) (0,3) (1,2) (1,3) (2,3): Pauli index and block coefficients of K
    const int pm[6] = {0, 0, 0, 1, 1, 2}, pn[6] = {1, 2, 3, 2, 3, 3};
    const int pl[6] = {0, 1, 2, 2, 1, 0};
    const double s0[6] = {1, 1, 1, -1, 1, -1};
    const double s1[6] = {-1, -1, -1, -1, 1, -1};
    const cx<double> ic2 = mk(0.0, 0.5 * csw);
    for (int pq = 0; pq < 6; ++pq) {
        const int mu = pm[pq], nu = pn[pq];
        M3 J;
        {
            M3 K;
            for (int q = 0; q < 9; ++q) K.a[q] = ic2 * (s0[pq] * L[0][pl[pq]].a[q] + s1[pq] * L[1][pl[pq]].a[q]);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    const cx<double> kij = K.a[3 * i + j], kji = K.a[3 * j + i];
                    J.a[3 * i + j] = mk((kij.re - kji.re) / 8.0, (kij.im + kji.im) / 8.0);
                }
        }
        const int xpm = step<+1>(g, y, mu), xpn = step<+1>(g, y, nu);
        const int xmm = step<-1>(g, y, mu), xmn = step<-1>(g, y, nu);
        const int xmm_pn = step<+1>(g, xmm, nu), xmm_mn = step<-1>(g, xmm, nu), xpm_mn = step<-1>(g, xpm, nu);
        // leaves as (direction, site, dagger) x 4, in product order (clover_build.h)
        const int lv[4][4][3] = {
            {{mu, y, 0}, {nu, xpm, 0}, {mu, xpn, 1}, {nu, y, 1}},
            {{nu, y, 0}, {mu, xmm_pn, 1}, {nu, xmm, 1}, {mu, xmm, 0}},
            {{mu, xmm, 1}, {nu, xmm_mn, 1}, {mu, xmm_mn, 0}, {nu, xmn, 0}},
            {{nu, xmn, 1}, {mu, xmn, 0}, {nu, xpm_mn, 0}, {mu, y, 1}}};
        for (int lf = 0; lf < 4; ++lf) {
            M3 f[4];
            for (int p = 0; p < 4; ++p) {
                f[p] = ld(U, g, lv[lf][p][0], lv[lf][p][1]);
                if (lv[lf][p][2]) f[p] = dag(f[p]);
            }
            for (int p = 0; p < 4; ++p) {
                // leaf = A X B with A = f[0..p-1], B = f[p+1..3]; Z = B J A
                M3 Z = J;
                for (int q = 0; q < p; ++q) Z = mul(Z, f[q]);
                for (int q = 3; q > p; --q) Z = mul(f[q], Z);
                add(lv[lf][p][0], lv[lf][p][1], lv[lf][p][2] ? Z : dag(Z));
            }
        }
    }
}

}  // namespace ddwc

// Clover field strength and the packed clover term of one site (setup code, shared by
// the device kernel and host-side checks).
#pragma once
#include "ddwc_device.h"

namespace ddwc {

// Neighbour of an arbitrary internal site (decodes it first).
template <int DIR>
DDWC_HD int step(const Geom& g, int s, int mu) {
    Site S = decode(g, s);
    bool in;
    int bc;
    return neighbour<DIR>(g, s, S, mu, in, bc);
}

struct M3 {
    cx<double> a[9];
};

DDWC_HD M3 ld(const cx<double>* U, const Geom& g, int mu, int s) {
    M3 m;
    for (int k = 0; k < 9; ++k) m.a[k] = U[((size_t)mu * 9 + k) * g.V + s];
    return m;
}
DDWC_HD M3 mul(const M3& x, const M3& y) {
    M3 z;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cx<double> t = mk(0.0, 0.0);
            for (int k = 0; k < 3; ++k) t = t + x.a[3 * i + k] * y.a[3 * k + j];
            z.a[3 * i + j] = t;
        }
    return z;
}
DDWC_HD M3 dag(const M3& x) {
    M3 z;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) z.a[3 * i + j] = mk(x.a[3 * j + i].re, -x.a[3 * j + i].im);
    return z;
}

// Fhat_{mu nu}(s) = (Q - Q^+)/8 from the four plaquette leaves at s (no boundary signs).
DDWC_HD M3 field_strength(const Geom& g, const cx<double>* U, int s, int mu, int nu) {
    int xpm = step<+1>(g, s, mu), xpn = step<+1>(g, s, nu);
    int xmm = step<-1>(g, s, mu), xmn = step<-1>(g, s, nu);
    int xmm_pn = step<+1>(g, xmm, nu), xmm_mn = step<-1>(g, xmm, nu), xpm_mn = step<-1>(g, xpm, nu);
    M3 q1 = mul(mul(ld(U, g, mu, s), ld(U, g, nu, xpm)), mul(dag(ld(U, g, mu, xpn)), dag(ld(U, g, nu, s))));
    M3 q2 = mul(mul(ld(U, g, nu, s), dag(ld(U, g, mu, xmm_pn))), mul(dag(ld(U, g, nu, xmm)), ld(U, g, mu, xmm)));
    M3 q3 = mul(mul(dag(ld(U, g, mu, xmm)), dag(ld(U, g, nu, xmm_mn))), mul(ld(U, g, mu, xmm_mn), ld(U, g, nu, xmn)));
    M3 q4 = mul(mul(dag(ld(U, g, nu, xmn)), ld(U, g, mu, xmn)), mul(ld(U, g, nu, xpm_mn), dag(ld(U, g, mu, s))));
    M3 F;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cx<double> q = q1.a[3 * i + j] + q2.a[3 * i + j] + q3.a[3 * i + j] + q4.a[3 * i + j];
            cx<double> qt = q1.a[3 * j + i] + q2.a[3 * j + i] + q3.a[3 * j + i] + q4.a[3 * j + i];
            F.a[3 * i + j] = mk((q.re - qt.re) / 8.0, (q.im + qt.im) / 8.0);
        }
    return F;
}

// Clover term in the chiral basis: sigma_{0k} = diag(s_k, -s_k), sigma_{jk} = -eps_{jkl} diag(s_l, s_l),
// so C = (i c_sw / 2) sum_l diag(s_l x E_l, s_l x E'_l) with
// E = (F01 - F23, F02 + F13, F03 - F12), E' = -(F01 + F23, F02 - F13, F03 + F12).

// The 72 packed reals of the clover term at site s (layout of ddwc_device.h).
// Chiral basis: sigma_{0k} = diag(s_k, -s_k), sigma_{jk} = -eps_{jkl} diag(s_l, s_l), so
// C = (i c_sw / 2) sum_l diag(s_l x E_l, s_l x E'_l) with
// E = (F01 - F23, F02 + F13, F03 - F12), E' = -(F01 + F23, F02 - F13, F03 + F12).
DDWC_HD void clover_site(const Geom& g, const cx<double>* U, double csw, int s, double a[72]) {
    M3 F01 = field_strength(g, U, s, 0, 1), F02 = field_strength(g, U, s, 0, 2), F03 = field_strength(g, U, s, 0, 3);
    M3 F12 = field_strength(g, U, s, 1, 2), F13 = field_strength(g, U, s, 1, 3), F23 = field_strength(g, U, s, 2, 3);
    for (int blk = 0; blk < 2; ++blk) {
        M3 E1, E2, E3;
        for (int k = 0; k < 9; ++k) {
            if (blk == 0) {
                E1.a[k] = F01.a[k] - F23.a[k];
                E2.a[k] = F02.a[k] + F13.a[k];
                E3.a[k] = F03.a[k] - F12.a[k];
            } else {
                E1.a[k] = -(F01.a[k] + F23.a[k]);
                E2.a[k] = -(F02.a[k] - F13.a[k]);
                E3.a[k] = -(F03.a[k] + F12.a[k]);
            }
        }
        cx<double> M[6][6];
        const cx<double> ic2 = mk(0.0, 0.5 * csw);
        for (int a1 = 0; a1 < 3; ++a1)
            for (int b1 = 0; b1 < 3; ++b1) {
                int k = 3 * a1 + b1;
                M[a1][b1] = ic2 * E3.a[k];
                M[3 + a1][3 + b1] = -(ic2 * E3.a[k]);
                M[a1][3 + b1] = ic2 * (E1.a[k] - times_i(E2.a[k]));
                M[3 + a1][b1] = ic2 * (E1.a[k] + times_i(E2.a[k]));
            }
        for (int i = 0; i < 6; ++i) a[6 * blk + i] = M[i][i].re;
        int k = 0;
        for (int i = 0; i < 6; ++i)
            for (int j = i + 1; j < 6; ++j) {
                a[12 + 30 * blk + 2 * k] = M[i][j].re;
                a[12 + 30 * blk + 2 * k + 1] = M[i][j].im;
                ++k;
            }
    }
}

}  // namespace ddwc

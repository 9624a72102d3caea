// Even-odd (red-black site parity) helpers.  With every Schwarz block extent even, the
// sites of a block are stored parity-major, so the even (odd) sites of all blocks form a
// half field of V/2 sites: half index i = B * Vb/2 + h for the h-th site of parity p in
// block B, full index s = B * Vb + p * Vb/2 + h.  Half fields keep the colour-major block
// order, so black blocks are the first half of a half field too.
//
// With A = 4 + m + C the site-diagonal part and H the hopping sum (D = A - H/2), the
// operator on even sites after eliminating the odd ones is
//     Mee = A_ee - D_eo A_oo^-1 D_oe = A_ee - 1/4 H_eo A_oo^-1 H_oe,
// and D x = b becomes Mee x_e = b_e + 1/2 H_eo A_oo^-1 b_o, x_o = A_oo^-1 (b_o + 1/2 H_oe x_e).
// Restricting H to hops inside a block gives the same structure for the Dirichlet
// block operators D_k.
#pragma once
#include "ddwc_device.h"

namespace ddwc {

DDWC_HD unsigned half_index(const Geom& g, unsigned s, int& p) {
    const unsigned B = s / (unsigned)g.Vb, loc = s - B * (unsigned)g.Vb;
    p = loc >= (unsigned)g.hvb;
    return B * (unsigned)g.hvb + loc - (unsigned)p * g.hvb;
}

DDWC_HD unsigned full_index(const Geom& g, unsigned i, int p) {
    const unsigned B = i / (unsigned)g.hvb;
    return i + (B + (unsigned)p) * (unsigned)g.hvb;
}

// Half-field neighbour-table entry of full-table entry e (sign kept).
DDWC_HD int half_entry(const Geom& g, int e) {
    int p;
    const unsigned t = e < 0 ? (unsigned)~e : (unsigned)e;
    const int h = (int)half_index(g, t, p);
    return e < 0 ? ~h : h;
}

// Inverse of the Hermitian positive definite 6x6 block (shift + K) in packed form
// (6 real diagonal entries d, 15 complex upper entries o in row order), by Cholesky
// A = L L^+, then A^-1 = L^-+ L^-1.  Returns the inverse in the same packing.
DDWC_HD void herm6_inverse(const double* d, const double* o, double shift, double* dinv, double* oinv) {
    cx<double> A[6][6];
    int k = 0;
    for (int i = 0; i < 6; ++i) {
        A[i][i] = mk(shift + d[i], 0.0);
        for (int j = i + 1; j < 6; ++j) {
            A[i][j] = mk(o[2 * k], o[2 * k + 1]);
            A[j][i] = mk(o[2 * k], -o[2 * k + 1]);
            ++k;
        }
    }
    cx<double> L[6][6];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) L[i][j] = mk(0.0, 0.0);
    for (int j = 0; j < 6; ++j) {
        double djj = A[j][j].re;
        for (int q = 0; q < j; ++q) djj -= L[j][q].re * L[j][q].re + L[j][q].im * L[j][q].im;
        const double ljj = sqrt(djj);
        L[j][j] = mk(ljj, 0.0);
        for (int i = j + 1; i < 6; ++i) {
            cx<double> t = A[i][j];
            for (int q = 0; q < j; ++q) t = t - L[i][q] * mk(L[j][q].re, -L[j][q].im);
            L[i][j] = mk(t.re / ljj, t.im / ljj);
        }
    }
    cx<double> M[6][6];  // L^-1, lower triangular
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) M[i][j] = mk(0.0, 0.0);
    for (int i = 0; i < 6; ++i) {
        M[i][i] = mk(1.0 / L[i][i].re, 0.0);
        for (int j = 0; j < i; ++j) {
            cx<double> t = mk(0.0, 0.0);
            for (int q = j; q < i; ++q) t = t + L[i][q] * M[q][j];
            M[i][j] = mk(-t.re / L[i][i].re, -t.im / L[i][i].re);
        }
    }
    k = 0;
    for (int i = 0; i < 6; ++i) {
        double di = 0;
        for (int q = i; q < 6; ++q) di += M[q][i].re * M[q][i].re + M[q][i].im * M[q][i].im;
        dinv[i] = di;
        for (int j = i + 1; j < 6; ++j) {
            cx<double> t = mk(0.0, 0.0);
            for (int q = j; q < 6; ++q) t = t + conj_mul(M[q][i], M[q][j]);
            oinv[2 * k] = t.re;
            oinv[2 * k + 1] = t.im;
            ++k;
        }
    }
}

// ln det of the Hermitian positive definite 6x6 block (shift + K) (packing of herm6_inverse),
// from its Cholesky factor: 2 sum_j ln L_jj.  Returns NaN if the block is not positive definite.
DDWC_HD double herm6_logdet(const double* d, const double* o, double shift) {
    cx<double> A[6][6];
    int k = 0;
    for (int i = 0; i < 6; ++i) {
        A[i][i] = mk(shift + d[i], 0.0);
        for (int j = i + 1; j < 6; ++j) {
            A[i][j] = mk(o[2 * k], o[2 * k + 1]);
            A[j][i] = mk(o[2 * k], -o[2 * k + 1]);
            ++k;
        }
    }
    cx<double> L[6][6];
    double ld = 0;
    for (int j = 0; j < 6; ++j) {
        double djj = A[j][j].re;
        for (int q = 0; q < j; ++q) djj -= L[j][q].re * L[j][q].re + L[j][q].im * L[j][q].im;
        if (!(djj > 0)) return NAN;
        const double ljj = sqrt(djj);
        ld += 2.0 * log(ljj);
        L[j][j] = mk(ljj, 0.0);
        for (int i = j + 1; i < 6; ++i) {
            cx<double> t = A[i][j];
            for (int q = 0; q < j; ++q) t = t - L[i][q] * mk(L[j][q].re, -L[j][q].im);
            L[i][j] = mk(t.re / ljj, t.im / ljj);
        }
    }
    return ld;
}

// out = (shift + A) v for the packed pair of Hermitian 6x6 blocks a[72] (layout of ddwc_device.h).
DDWC_HD void packed_apply(const double a[72], double shift, const cx<double> v[12], cx<double> out[12]) {
    for (int blk = 0; blk < 2; ++blk) {
        const cx<double>* x = v + 6 * blk;
        cx<double>* y = out + 6 * blk;
        for (int i = 0; i < 6; ++i) y[i] = mk((shift + a[6 * blk + i]) * x[i].re, (shift + a[6 * blk + i]) * x[i].im);
        int k = 0;
        for (int i = 0; i < 6; ++i)
            for (int j = i + 1; j < 6; ++j) {
                const cx<double> aij = mk(a[12 + 30 * blk + 2 * k], a[12 + 30 * blk + 2 * k + 1]);
                cmadd(y[i], aij, x[j]);
                cjmadd(y[j], aij, x[i]);
                ++k;
            }
    }
}

// Packed inverse of A = (4 + m) + C at one site: a = packed clover (72 reals), mass4 = 4 + m.
DDWC_HD void clover_inverse_site(const double a[72], double mass4, double out[72]) {
    for (int blk = 0; blk < 2; ++blk) herm6_inverse(a + 6 * blk, a + 12 + 30 * blk, mass4, out + 6 * blk, out + 12 + 30 * blk);
}

}  // namespace ddwc

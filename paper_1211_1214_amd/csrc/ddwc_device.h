// Device-side building blocks of the ddwc library (gfx950).
//
// Internal site order is block-major: site s = ((c * NBc + rank) * Vb) + local,
// with c the Schwarz colour (black = 0), rank the block's number among the blocks of
// that colour and local the site inside the block: lexicographic, or, when every block
// extent is even, parity-major (the even sites of the block, then the odd ones, each
// in lexicographic order) so that even and odd half-vectors are contiguous per block.  Black sites are
// the first half of every field, and each block's sites are contiguous, so a
// workgroup that owns one block reads it with unit stride.
//
// Fields are SoA, site fastest, in 16-byte words:
//   spinor  [nrhs][NCW][V] words   FP64: one complex per double2 (NCW = 12)
//                                  FP32: two complex per float4  (NCW = 6)
//   links   [4][9][V] complex      (row-major 3x3, U_mu(x) from x to x + mu)
//   clover  [NKW][V] words of the 72 reals of two Hermitian 6x6 blocks
//           (chiral spin blocks {0,1} and {2,3}); FP64 NKW = 36, FP32 NKW = 18.
//           Reals 0..5: diagonal of block 0, 6..11: diagonal of block 1,
//           12..41: upper off-diagonal of block 0 as (re, im) in row order
//           (0,1),(0,2),...,(0,5),(1,2),...,(4,5), 42..71: same for block 1.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define DDWC_HD __host__ __device__ __forceinline__

namespace ddwc {

template <class R>
struct cx {
    R re, im;
};

template <class R>
DDWC_HD cx<R> mk(R a, R b) {
    cx<R> z;
    z.re = a;
    z.im = b;
    return z;
}
template <class R>
DDWC_HD cx<R> operator+(cx<R> a, cx<R> b) { return mk(a.re + b.re, a.im + b.im); }
template <class R>
DDWC_HD cx<R> operator-(cx<R> a, cx<R> b) { return mk(a.re - b.re, a.im - b.im); }
template <class R>
DDWC_HD cx<R> operator-(cx<R> a) { return mk(-a.re, -a.im); }
template <class R>
DDWC_HD cx<R> operator*(cx<R> a, cx<R> b) {
    return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <class R>
DDWC_HD cx<R> operator*(R s, cx<R> a) { return mk(s * a.re, s * a.im); }
template <class R>
DDWC_HD cx<R> conj_mul(cx<R> a, cx<R> b) {  // conj(a) * b
    return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
template <class R>
DDWC_HD cx<R> times_i(cx<R> a) { return mk(-a.im, a.re); }
template <class R>
DDWC_HD cx<R> times_mi(cx<R> a) { return mk(a.im, -a.re); }

DDWC_HD float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
DDWC_HD double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

// acc += a b and acc += conj(a) b as explicit fused multiply-adds.
template <class R>
DDWC_HD void cmadd(cx<R>& acc, cx<R> a, cx<R> b) {
    acc.re = fmad(a.re, b.re, fmad(-a.im, b.im, acc.re));
    acc.im = fmad(a.re, b.im, fmad(a.im, b.re, acc.im));
}
template <class R>
DDWC_HD void cjmadd(cx<R>& acc, cx<R> a, cx<R> b) {
    acc.re = fmad(a.re, b.re, fmad(a.im, b.im, acc.re));
    acc.im = fmad(a.re, b.im, fmad(-a.im, b.re, acc.im));
}

// ------------------------------------------------------------------ geometry
struct Geom {
    int L[4];      // T, L1, L2, L3
    int b[4];      // block extents
    int nb[4];     // blocks per direction
    int lstr[4];   // lexicographic stride of a unit step inside a block
    int V, Vb, NB, NBc, nb3h;
    int tbc;       // time boundary factor (-1 antiperiodic, +1 periodic)
    int eo;        // 1 when every block extent is even: sites inside a block are ordered
                   // parity-major (even sites first), parity = (x0+x1+x2+x3) mod 2
    int hvb;       // Vb / 2
};

// Geometry of a T x L1 x L2 x L3 lattice split into blocks blk (extents already validated).
inline Geom make_geom(const int lat[4], const int blk[4], int time_bc) {
    Geom g;
    for (int mu = 0; mu < 4; ++mu) {
        g.L[mu] = lat[mu];
        g.b[mu] = blk[mu];
        g.nb[mu] = lat[mu] / blk[mu];
    }
    g.lstr[3] = 1;
    g.lstr[2] = g.b[3];
    g.lstr[1] = g.b[3] * g.b[2];
    g.lstr[0] = g.b[3] * g.b[2] * g.b[1];
    g.V = lat[0] * lat[1] * lat[2] * lat[3];
    g.Vb = g.b[0] * g.b[1] * g.b[2] * g.b[3];
    g.NB = g.V / g.Vb;
    g.NBc = g.NB / 2;
    g.nb3h = g.nb[3] / 2;
    g.tbc = time_bc;
    g.eo = (blk[0] % 2 == 0 && blk[1] % 2 == 0 && blk[2] % 2 == 0 && blk[3] % 2 == 0) ? 1 : 0;
    g.hvb = g.Vb / 2;
    return g;
}

struct Site {
    int l[4];  // coordinates inside the block
    int n[4];  // block coordinates
    int c;     // colour
};

DDWC_HD Site decode(const Geom& g, int s) {
    Site S;
    int loc = s % g.Vb;
    int B = s / g.Vb;
    int p = 0;
    if (g.eo) {
        // parity-major: loc = p * Vb/2 + (lexicographic index >> 1); rows of even length b3
        // alternate parity, so the lexicographic index is 2h or 2h + 1
        p = loc / g.hvb;
        loc = 2 * (loc - p * g.hvb);
    }
    S.l[3] = loc % g.b[3];
    loc /= g.b[3];
    S.l[2] = loc % g.b[2];
    loc /= g.b[2];
    S.l[1] = loc % g.b[1];
    S.l[0] = loc / g.b[1];
    if (g.eo && ((S.l[0] + S.l[1] + S.l[2] + S.l[3]) & 1) != p) S.l[3] += 1;
    S.c = B / g.NBc;
    int r = B % g.NBc;
    int h = r % g.nb3h;
    r /= g.nb3h;
    S.n[2] = r % g.nb[2];
    r /= g.nb[2];
    S.n[1] = r % g.nb[1];
    S.n[0] = r / g.nb[1];
    S.n[3] = 2 * h + ((S.c + S.n[0] + S.n[1] + S.n[2]) & 1);
    return S;
}

DDWC_HD int block_base(const Geom& g, const int n[4]) {
    int c = (n[0] + n[1] + n[2] + n[3]) & 1;
    int r = ((n[0] * g.nb[1] + n[1]) * g.nb[2] + n[2]) * g.nb3h + (n[3] >> 1);
    return (c * g.NBc + r) * g.Vb;
}

DDWC_HD int local_index(const Geom& g, const int l[4]) {
    const int lex = ((l[0] * g.b[1] + l[1]) * g.b[2] + l[2]) * g.b[3] + l[3];
    if (!g.eo) return lex;
    return ((l[0] + l[1] + l[2] + l[3]) & 1) * g.hvb + (lex >> 1);
}

// Neighbour of site s (decoded as S) one step forward (+1) or backward (-1) in mu.
// Sets inside = whether it lies in the same Schwarz block, and bc = the
// time-boundary factor of the hop.
template <int DIR>
DDWC_HD int neighbour(const Geom& g, int s, const Site& S, int mu, bool& inside, int& bc) {
    bc = 1;
    if (DIR > 0) {
        if (S.l[mu] < g.b[mu] - 1) {
            inside = true;
            int l[4] = {S.l[0], S.l[1], S.l[2], S.l[3]};
            l[mu] += 1;
            return (s - s % g.Vb) + local_index(g, l);
        }
        inside = false;
        int n[4] = {S.n[0], S.n[1], S.n[2], S.n[3]};
        int l[4] = {S.l[0], S.l[1], S.l[2], S.l[3]};
        l[mu] = 0;
        n[mu] = n[mu] + 1;
        if (n[mu] == g.nb[mu]) {
            n[mu] = 0;
            if (mu == 0) bc = g.tbc;
        }
        return block_base(g, n) + local_index(g, l);
    } else {
        if (S.l[mu] > 0) {
            inside = true;
            int l[4] = {S.l[0], S.l[1], S.l[2], S.l[3]};
            l[mu] -= 1;
            return (s - s % g.Vb) + local_index(g, l);
        }
        inside = false;
        int n[4] = {S.n[0], S.n[1], S.n[2], S.n[3]};
        int l[4] = {S.l[0], S.l[1], S.l[2], S.l[3]};
        l[mu] = g.b[mu] - 1;
        n[mu] = n[mu] - 1;
        if (n[mu] < 0) {
            n[mu] = g.nb[mu] - 1;
            if (mu == 0) bc = g.tbc;
        }
        return block_base(g, n) + local_index(g, l);
    }
}

// The black face sites: range of the projector P.
DDWC_HD bool in_P(const Geom& g, const Site& S) {
    if (S.c != 0) return false;
    for (int mu = 0; mu < 4; ++mu)
        if (S.l[mu] == 0 || S.l[mu] == g.b[mu] - 1) return true;
    return false;
}

// Lexicographic (canonical) site index of a decoded internal site.
DDWC_HD int canonical_index(const Geom& g, const Site& S) {
    int x[4];
    for (int mu = 0; mu < 4; ++mu) x[mu] = S.n[mu] * g.b[mu] + S.l[mu];
    return ((x[0] * g.L[1] + x[1]) * g.L[2] + x[2]) * g.L[3] + x[3];
}

// ------------------------------------------------------------------ storage traits
template <class R>
struct Traits;

// Storage of one precision: `word` the 16-byte spinor word, `real` the arithmetic type,
// `link` the storage of a link entry, `kword` the clover word, `xs` the precision that
// accumulates a solver's solution.
template <>
struct Traits<double> {
    typedef double2 word;
    typedef double real;
    typedef double link;
    typedef double2 kword;
    typedef double xs;
    static constexpr int NCW = 12;  // spinor words per site
    static constexpr int NKW = 36;  // clover words per site
};
template <>
struct Traits<float> {
    typedef float4 word;
    typedef float real;
    typedef float link;
    typedef float4 kword;
    typedef float xs;
    static constexpr int NCW = 6;
    static constexpr int NKW = 18;
};

// FP16 storage with FP32 arithmetic: a spinor is three words of eight halves (four complex)
// scaled by one FP32 factor per site (its largest component modulus), kept in a plane of
// floats after the word planes; links are plain halves (|U_ij| <= 1); the clover stays FP32.
struct H16 {};
typedef _Float16 f16;
struct __attribute__((aligned(16))) hw16 {
    f16 h[8];
};
template <>
struct Traits<H16> {
    typedef hw16 word;
    typedef float real;
    typedef f16 link;
    typedef float4 kword;
    typedef float xs;
    static constexpr int NCW = 3;
    static constexpr int NKW = 18;
};

// Element i of an array whose byte size stays below 4 GiB: the byte offset is formed in
// 32 bits, so a load is a uniform base plus a 32-bit per-lane offset.
template <class T>
DDWC_HD const T& at(const T* base, unsigned i) {
    return *(const T*)((const char*)base + i * (unsigned)sizeof(T));
}
template <class T>
DDWC_HD T& at(T* base, unsigned i) {
    return *(T*)((char*)base + i * (unsigned)sizeof(T));
}

DDWC_HD void load_spinor(const double2* __restrict__ f, unsigned V, unsigned s, cx<double> p[12]) {
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        double2 w = at(f + (size_t)c * V, s);
        p[c] = mk(w.x, w.y);
    }
}
DDWC_HD void load_spinor(const float4* __restrict__ f, unsigned V, unsigned s, cx<float> p[12]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        float4 w = at(f + (size_t)k * V, s);
        p[2 * k] = mk(w.x, w.y);
        p[2 * k + 1] = mk(w.z, w.w);
    }
}
DDWC_HD void store_spinor(double2* __restrict__ f, unsigned V, unsigned s, const cx<double> p[12]) {
#pragma unroll
    for (int c = 0; c < 12; ++c) at(f + (size_t)c * V, s) = make_double2(p[c].re, p[c].im);
}
DDWC_HD void store_spinor(float4* __restrict__ f, unsigned V, unsigned s, const cx<float> p[12]) {
#pragma unroll
    for (int k = 0; k < 6; ++k)
        at(f + (size_t)k * V, s) = make_float4(p[2 * k].re, p[2 * k].im, p[2 * k + 1].re, p[2 * k + 1].im);
}

template <class R, class L>
DDWC_HD void load_link(const cx<L>* __restrict__ U, unsigned V, int mu, unsigned s, cx<R> u[9]) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const cx<L> w = at(U + (size_t)(mu * 9 + k) * V, s);
        u[k] = mk((R)w.re, (R)w.im);
    }
}

// Site-major links [n][4][9]: the four forward links of a site are one contiguous record, so the
// lanes of a site (RHS-innermost kernels) read whole cache lines at once.
template <bool SITE_MAJOR, class R, class L>
DDWC_HD void load_link_l(const cx<L>* __restrict__ U, unsigned V, int mu, unsigned s, cx<R> u[9]) {
    if (!SITE_MAJOR) {
        load_link(U, V, mu, s, u);
        return;
    }
    const cx<L>* p = U + ((size_t)s * 4 + mu) * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const cx<L> w = p[k];
        u[k] = mk((R)w.re, (R)w.im);
    }
}

// Link layouts of the hop kernels: LK_ENTRY entry-major [4][9][n] (forward links at s from Uf,
// backward links at the neighbour t from Ub), LK_SITE site-major [n][4][9] (same roles),
// LK_OWN own-site records [n][8][9] of Uf: for each site the eight links its hops use, d = 2 mu
// holding U_mu(x) and d = 2 mu + 1 holding U_mu(x - mu), so that every hop reads its link from
// the site's own contiguous record (no gather of backward links).
enum LinkLayout { LK_ENTRY = 0, LK_SITE = 1, LK_OWN = 2 };

template <int LK, class R, class L>
DDWC_HD void hop_link(const cx<L>* __restrict__ Uf, const cx<L>* __restrict__ Ub, unsigned n, int d, unsigned s,
                      unsigned t, cx<R> u[9]) {
    if (LK == LK_OWN) {
        const cx<L>* p = Uf + ((size_t)s * 8 + d) * 9;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const cx<L> w = p[k];
            u[k] = mk((R)w.re, (R)w.im);
        }
        return;
    }
    if (d & 1)
        load_link_l<LK == LK_SITE>(Ub, n, d >> 1, t, u);
    else
        load_link_l<LK == LK_SITE>(Uf, n, d >> 1, s, u);
}

// FP16 spinors: words k = 0..2 hold complex 4k .. 4k + 3; the scale plane follows the three
// word planes of the field (f is the field base, `stride` its plane length).
DDWC_HD float* scale_plane(hw16* f, unsigned stride) { return (float*)(f + 3 * (size_t)stride); }
DDWC_HD const float* scale_plane(const hw16* f, unsigned stride) { return (const float*)(f + 3 * (size_t)stride); }
DDWC_HD void load_spinor(const hw16* __restrict__ f, unsigned stride, unsigned s, cx<float> p[12]) {
    const float sc = at(scale_plane(f, stride), s);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const hw16 w = at(f + (size_t)k * stride, s);
#pragma unroll
        for (int q = 0; q < 4; ++q) p[4 * k + q] = mk(sc * (float)w.h[2 * q], sc * (float)w.h[2 * q + 1]);
    }
}
DDWC_HD void store_spinor(hw16* __restrict__ f, unsigned stride, unsigned s, const cx<float> p[12]) {
    float m = 0.f;
#pragma unroll
    for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf(p[c].re), fabsf(p[c].im)));
    const float inv = m > 0.f ? 1.f / m : 0.f;
    at(scale_plane(f, stride), s) = m;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        hw16 w;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            w.h[2 * q] = (f16)(inv * p[4 * k + q].re);
            w.h[2 * q + 1] = (f16)(inv * p[4 * k + q].im);
        }
        at(f + (size_t)k * stride, s) = w;
    }
}

// The 36 reals of chiral block `blk` of the clover term at site s:
// d[0..5] = diagonal, o[0..29] = upper off-diagonal (re, im) in row order.
DDWC_HD void load_clover_block(const double2* __restrict__ K, unsigned V, unsigned s, int blk, double d[6],
                                                  double o[30]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double2 w = at(K + (size_t)(3 * blk + k) * V, s);
        d[2 * k] = w.x;
        d[2 * k + 1] = w.y;
    }
#pragma unroll
    for (int k = 0; k < 15; ++k) {
        double2 w = at(K + (size_t)(6 + 15 * blk + k) * V, s);
        o[2 * k] = w.x;
        o[2 * k + 1] = w.y;
    }
}
// FP32: reals 0..11 are words 0..2; block 0 off-diagonal reals 12..41 start in word 3,
// block 1 reals 42..71 start at word 10 offset 2.  Load the 9 words that cover a block.
DDWC_HD void load_clover_block(const float4* __restrict__ K, unsigned V, unsigned s, int blk, float d[6],
                                                  float o[30]) {
    float w[40];
    const int w0 = blk == 0 ? 3 : 10;  // first word holding off-diagonal reals of this block
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        float4 q = at(K + (size_t)(w0 + k) * V, s);
        w[4 * k] = q.x;
        w[4 * k + 1] = q.y;
        w[4 * k + 2] = q.z;
        w[4 * k + 3] = q.w;
    }
    const int sh = blk == 0 ? 0 : 2;  // reals 42.. start at offset 2 of word 10
#pragma unroll
    for (int k = 0; k < 30; ++k) o[k] = w[sh + k];
    // diagonal reals 6*blk .. 6*blk+5 live in words 0..2
    float4 q0 = at(K + (size_t)(blk == 0 ? 0 : 1) * V, s);
    float4 q1 = at(K + (size_t)(blk == 0 ? 1 : 2) * V, s);
    if (blk == 0) {
        d[0] = q0.x; d[1] = q0.y; d[2] = q0.z; d[3] = q0.w; d[4] = q1.x; d[5] = q1.y;
    } else {
        d[0] = q0.z; d[1] = q0.w; d[2] = q1.x; d[3] = q1.y; d[4] = q1.z; d[5] = q1.w;
    }
}

// y = (4 + m) psi + C psi + hsc * y with the two packed Hermitian 6x6 blocks, one block at
// a time (y holds the accumulated hop terms on entry, hsc = -1/2; hsc = 0 ignores them).
template <class R>
DDWC_HD void apply_diag(const typename Traits<R>::word* __restrict__ K, unsigned V, unsigned s, R mass4,
                        const cx<R> p[12], cx<R> y[12], R hsc) {
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
        R d[6], o[30];
        load_clover_block(K, V, s, blk, d, o);
        const cx<R>* v = p + 6 * blk;
        cx<R>* w = y + 6 * blk;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const R di = mass4 + d[i];
            w[i] = mk(fmad(di, v[i].re, hsc * w[i].re), fmad(di, v[i].im, hsc * w[i].im));
        }
        int k = 0;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
#pragma unroll
            for (int j = i + 1; j < 6; ++j) {
                const cx<R> aij = mk(o[2 * k], o[2 * k + 1]);
                cmadd(w[i], aij, v[j]);
                cjmadd(w[j], aij, v[i]);
                ++k;
            }
        }
    }
}

// One hop term in the chiral basis: acc += (1 - g_mu) U q (DIR = +1) or
// (1 + g_mu) U^+ q (DIR = -1), through the spin-projected half spinor
// h = (h0, h1) (2 spins x 3 colours):
//   mu = 0:  h = q_u -+ q_l         lower spins of the term = +- k
//   mu = k:  h = q_u +- i s_k q_l   lower spins = -+ i s_k k       (k = U h or U^+ h)
// MU and DIR are compile-time, so each direction is straight-line code.
template <class R, int MU, int DIR>
DDWC_HD void hop_term(const cx<R> u[9], const cx<R> q[12], cx<R> acc[12]) {
    cx<R> h0[3], h1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cx<R> p0 = q[a], p1 = q[3 + a], p2 = q[6 + a], p3 = q[9 + a];
        if (MU == 0) {
            h0[a] = DIR > 0 ? p0 + p2 : p0 - p2;
            h1[a] = DIR > 0 ? p1 + p3 : p1 - p3;
        } else if (MU == 1) {
            h0[a] = DIR > 0 ? p0 + times_i(p3) : p0 - times_i(p3);
            h1[a] = DIR > 0 ? p1 + times_i(p2) : p1 - times_i(p2);
        } else if (MU == 2) {
            h0[a] = DIR > 0 ? p0 + p3 : p0 - p3;
            h1[a] = DIR > 0 ? p1 - p2 : p1 + p2;
        } else {
            h0[a] = DIR > 0 ? p0 + times_i(p2) : p0 - times_i(p2);
            h1[a] = DIR > 0 ? p1 - times_i(p3) : p1 + times_i(p3);
        }
    }
    cx<R> k0[3], k1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        k0[a] = mk(R(0), R(0));
        k1[a] = mk(R(0), R(0));
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if (DIR > 0) {
                cmadd(k0[a], u[3 * a + b], h0[b]);
                cmadd(k1[a], u[3 * a + b], h1[b]);
            } else {
                cjmadd(k0[a], u[3 * b + a], h0[b]);
                cjmadd(k1[a], u[3 * b + a], h1[b]);
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        acc[a] = acc[a] + k0[a];
        acc[3 + a] = acc[3 + a] + k1[a];
        cx<R> l0, l1;
        if (MU == 0) {
            l0 = DIR > 0 ? k0[a] : -k0[a];
            l1 = DIR > 0 ? k1[a] : -k1[a];
        } else if (MU == 1) {
            l0 = DIR > 0 ? times_mi(k1[a]) : times_i(k1[a]);
            l1 = DIR > 0 ? times_mi(k0[a]) : times_i(k0[a]);
        } else if (MU == 2) {
            l0 = DIR > 0 ? -k1[a] : k1[a];
            l1 = DIR > 0 ? k0[a] : -k0[a];
        } else {
            l0 = DIR > 0 ? times_mi(k0[a]) : times_i(k0[a]);
            l1 = DIR > 0 ? times_i(k1[a]) : times_mi(k1[a]);
        }
        acc[6 + a] = acc[6 + a] + l0;
        acc[9 + a] = acc[9 + a] + l1;
    }
}

// Direction d = 2 mu + (backward ? 1 : 0), chosen at run time (uniform across the wave).
template <class R>
DDWC_HD void hop_dispatch(int d, const cx<R> u[9], const cx<R> q[12], cx<R> acc[12]) {
    switch (d) {
        case 0: hop_term<R, 0, +1>(u, q, acc); break;
        case 1: hop_term<R, 0, -1>(u, q, acc); break;
        case 2: hop_term<R, 1, +1>(u, q, acc); break;
        case 3: hop_term<R, 1, -1>(u, q, acc); break;
        case 4: hop_term<R, 2, +1>(u, q, acc); break;
        case 5: hop_term<R, 2, -1>(u, q, acc); break;
        case 6: hop_term<R, 3, +1>(u, q, acc); break;
        default: hop_term<R, 3, -1>(u, q, acc); break;
    }
}

// Neighbour-table entry of site s in direction d = 2 mu + (backward ? 1 : 0): the
// neighbour's internal index, bitwise-negated when the hop crosses an antiperiodic
// time boundary.
template <int DIR>
DDWC_HD int table_entry(const Geom& g, int s, const Site& S, int mu) {
    bool inside;
    int bc;
    const int t = neighbour<DIR>(g, s, S, mu, inside, bc);
    return bc < 0 ? ~t : t;
}

// Which hops a site operator includes.
enum HopSet { HOPS_NONE = 0, HOPS_ALL = 1, HOPS_INSIDE = 2, HOPS_CROSSING = 3 };

// acc = sum over the selected hops of site s of (1 -+ g_mu) W psi(neighbour), unscaled; a
// hop across an antiperiodic time boundary is subtracted.  The index space has length n
// (V for full fields, V/2 for even-odd half fields); nbr is its neighbour table [8][n];
// forward links are read from Uf at s, backward links from Ub at the neighbour.  Both
// index spaces are colour-major, so a neighbour lies in the same Schwarz block exactly
// when it lies in the same half.  `ndir` is 8; it is a run-time value so that the
// direction loop stays a loop and only one neighbour spinor and link are live at a time.
// PIPE 1: the next direction's spinor and link loads are issued before the current one is
// computed.  PIPE 2: the direction loop is unrolled (no pipelining): the spin algebra of each
// direction is then straight-line code instead of a switch whose merge copies the accumulator
// (24 moves per hop); for hop sets with a per-hop condition (inside / crossing), whose branches
// keep the scheduler from hoisting every direction's loads.  (With HOPS_ALL the unrolled loop
// hoists them all: 256 VGPRs.)
//
// Spinors may be stored RHS-innermost: the spinor of site t is element t * smul + sadd of
// component arrays sstride apart (RHS-major: smul = 1, sadd = 0, sstride = n).  Links are
// in the layout LK (LinkLayout; Uf's own-site records with LK_OWN).
// With LK_OWN the records may be a staged copy (in LDS) that starts at site `l0`: the record of
// s is then record s - l0 of Uf.  With nstr > 0 the neighbour table is a staged copy too,
// [8][nstr] entries starting at site l0.
template <class R, int HOPS, int PIPE, int LK = LK_ENTRY, class W, class L>
DDWC_HD void hop_sum(unsigned n, unsigned s, const W* __restrict__ in, const cx<L>* __restrict__ Uf,
                     const cx<L>* __restrict__ Ub, const int* __restrict__ nbr, cx<R> acc[12], int ndir,
                     unsigned smul = 1, unsigned sadd = 0, unsigned sstride = 0, unsigned l0 = 0,
                     unsigned nstr = 0) {
    if (sstride == 0) sstride = n;
    const unsigned sl = s - l0;  // record index of s (LK_OWN)
    const unsigned ns = nstr ? nstr : n, sn = nstr ? sl : s;  // table stride and index of s
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = mk(R(0), R(0));
    if (HOPS == HOPS_NONE) return;
    const bool s_black = s < n / 2;
    if (PIPE == 0 || PIPE == 2) {
#pragma unroll(PIPE == 2 ? 8 : 1)
        for (int d = 0; d < (PIPE == 2 ? 8 : ndir); ++d) {
            const int e = at(nbr + (size_t)d * ns, sn);
            const unsigned t = e < 0 ? (unsigned)~e : (unsigned)e;
            const bool inside = (t < n / 2) == s_black;
            const bool take = HOPS == HOPS_ALL || (HOPS == HOPS_INSIDE && inside) || (HOPS == HOPS_CROSSING && !inside);
            if (take) {
                cx<R> q[12], u[9];
                load_spinor(in, sstride, t * smul + sadd, q);
                hop_link<LK>(Uf, Ub, n, d, LK == LK_OWN ? sl : s, t, u);
                if (e < 0) {
#pragma unroll
                    for (int c = 0; c < 12; ++c) q[c] = -q[c];
                }
                hop_dispatch<R>(d, u, q, acc);
            }
        }
    } else {
        // all eight table entries first, then a software-pipelined direction loop: the
        // neighbour spinor and link of direction d + 1 are in flight while d is computed
        int ent[8];
#pragma unroll
        for (int d = 0; d < 8; ++d) ent[d] = at(nbr + (size_t)d * ns, sn);
        cx<R> q[12], u[9];
        {
            const int e = ent[0];
            const unsigned t0 = e < 0 ? (unsigned)~e : (unsigned)e;
            load_spinor(in, sstride, t0 * smul + sadd, q);
            hop_link<LK>(Uf, Ub, n, 0, LK == LK_OWN ? sl : s, t0, u);
        }
#pragma unroll 1
        for (int d = 0; d < ndir; ++d) {
            int e = ent[0];
#pragma unroll
            for (int k = 1; k < 8; ++k) e = d == k ? ent[k] : e;
            const unsigned t = e < 0 ? (unsigned)~e : (unsigned)e;
            const bool inside = (t < n / 2) == s_black;
            const bool take = HOPS == HOPS_ALL || (HOPS == HOPS_INSIDE && inside) || (HOPS == HOPS_CROSSING && !inside);
            cx<R> qn[12], un[9];
            if (d + 1 < ndir) {
                int en = ent[1];
#pragma unroll
                for (int k = 2; k < 8; ++k) en = d + 1 == k ? ent[k] : en;
                const unsigned tn = en < 0 ? (unsigned)~en : (unsigned)en;
                load_spinor(in, sstride, tn * smul + sadd, qn);
                hop_link<LK>(Uf, Ub, n, d + 1, LK == LK_OWN ? sl : s, tn, un);
            }
            if (take) {
                if (e < 0) {
#pragma unroll
                    for (int c = 0; c < 12; ++c) q[c] = -q[c];
                }
                hop_dispatch<R>(d, u, q, acc);
            }
#pragma unroll
            for (int c = 0; c < 12; ++c) q[c] = qn[c];
#pragma unroll
            for (int c = 0; c < 9; ++c) u[c] = un[c];
        }
    }
}

// y = [diag] (4+m+C) psi(s) - 1/2 sum over the selected hops, on full fields.  `in`
// points at one RHS, nbr is the neighbour table [8][V].
template <class R, bool DIAG, int HOPS, int PIPE = 0>
DDWC_HD void site_operator(const Geom& g, unsigned s, const typename Traits<R>::word* __restrict__ in,
                           const cx<R>* __restrict__ U, const typename Traits<R>::word* __restrict__ K,
                           const int* __restrict__ nbr, R mass4, cx<R> y[12], int ndir) {
    const unsigned V = g.V;
    hop_sum<R, HOPS, PIPE>(V, s, in, U, U, nbr, y, ndir);
    if (DIAG) {
        cx<R> c[12];
        load_spinor(in, V, s, c);
        apply_diag<R>(K, V, s, mass4, c, y, R(-0.5));
    } else {
#pragma unroll
        for (int c = 0; c < 12; ++c) y[c] = R(-0.5) * y[c];
    }
}

// ------------------------------------------------------------------ reductions
// Sum over the workgroup; every thread receives the total.  `lds` holds one
// double per wave; the order of the sums is fixed, so results are reproducible.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Workgroup sum with one barrier: `lds` (NV x 16 doubles) must not be the slot of the previous
// block_sum1 of the workgroup (alternate two slots), which all threads have finished reading
// before any of them reaches this barrier.
template <int NV>
__device__ __forceinline__ void block_sum1(double v[NV], double* lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0)
        for (int k = 0; k < NV; ++k) lds[k * 16 + wave] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double t = 0;
        for (int w = 0; w < nw; ++w) t += lds[k * 16 + w];
        v[k] = t;
    }
}

template <int NV>
__device__ __forceinline__ void block_sum(double v[NV], double* lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    __syncthreads();
    if (lane == 0)
        for (int k = 0; k < NV; ++k) lds[k * 16 + wave] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double t = 0;
        for (int w = 0; w < nw; ++w) t += lds[k * 16 + w];
        v[k] = t;
    }
}

// Per-RHS partial sums of a workgroup whose thread j holds values of RHS (g0 + j) mod nrhs
// (RHS-innermost work items): thread r < nrhs sums its RHS in a fixed order and writes
// part[(k * nrhs + r) * ntiles + tile].  Needs nrhs <= blockDim.x <= NT.  The values pass
// through LDS as T (float where every value is an FP32 sum converted to double: exact).
template <int NV, int NT = 256, class T = double>
__device__ __forceinline__ void seg_partials(const double v[NV], double* part, int ntiles, int tile, unsigned g0,
                                             int nrhs) {
    __shared__ T lds[NV][NT];
#pragma unroll
    for (int k = 0; k < NV; ++k) lds[k][threadIdx.x] = (T)v[k];
    __syncthreads();
    if ((int)threadIdx.x < nrhs) {
        const int r = threadIdx.x;
        const int j0 = (int)((r + nrhs - (int)(g0 % (unsigned)nrhs)) % nrhs);
        double acc[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) acc[k] = 0;
        for (int j = j0; j < (int)blockDim.x; j += nrhs)
#pragma unroll
            for (int k = 0; k < NV; ++k) acc[k] += (double)lds[k][j];
#pragma unroll
        for (int k = 0; k < NV; ++k) part[((size_t)k * nrhs + r) * ntiles + tile] = acc[k];
    }
}

// ------------------------------------------------------------------ per-site dot products (FP64 accumulate)
template <class R>
DDWC_HD void acc_dot(const cx<R> a[12], const cx<R> b[12], double& re, double& im) {
    // (a, b) = sum conj(a) b
    R sr = 0, si = 0;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        sr += a[c].re * b[c].re + a[c].im * b[c].im;
        si += a[c].re * b[c].im - a[c].im * b[c].re;
    }
    re += (double)sr;
    im += (double)si;
}

template <class R>
DDWC_HD double acc_nrm(const cx<R> a[12]) {
    R s = 0;
#pragma unroll
    for (int c = 0; c < 12; ++c) s += a[c].re * a[c].re + a[c].im * a[c].im;
    return (double)s;
}

}  // namespace ddwc

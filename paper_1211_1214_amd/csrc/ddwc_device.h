// Device-side building blocks of the ddwc library (gfx950).
//
// Internal site order is block-major: site s = ((c * NBc + rank) * Vb) + local,
// with c the Schwarz colour (black = 0), rank the block's number among the blocks of
// that colour and local the lexicographic site inside the block.  Black sites are
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

// ------------------------------------------------------------------ geometry
struct Geom {
    int L[4];      // T, L1, L2, L3
    int b[4];      // block extents
    int nb[4];     // blocks per direction
    int lstr[4];   // stride of a unit step inside a block (local index)
    int V, Vb, NB, NBc, nb3h;
    int tbc;       // time boundary factor (-1 antiperiodic, +1 periodic)
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
    S.l[3] = loc % g.b[3];
    loc /= g.b[3];
    S.l[2] = loc % g.b[2];
    loc /= g.b[2];
    S.l[1] = loc % g.b[1];
    S.l[0] = loc / g.b[1];
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
    return ((l[0] * g.b[1] + l[1]) * g.b[2] + l[2]) * g.b[3] + l[3];
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
            return s + g.lstr[mu];
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
            return s - g.lstr[mu];
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

template <>
struct Traits<double> {
    typedef double2 word;
    static constexpr int NCW = 12;  // spinor words per site
    static constexpr int NKW = 36;  // clover words per site
};
template <>
struct Traits<float> {
    typedef float4 word;
    static constexpr int NCW = 6;
    static constexpr int NKW = 18;
};

DDWC_HD void load_spinor(const double2* __restrict__ f, int V, int s, cx<double> p[12]) {
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        double2 w = f[(size_t)c * V + s];
        p[c] = mk(w.x, w.y);
    }
}
DDWC_HD void load_spinor(const float4* __restrict__ f, int V, int s, cx<float> p[12]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        float4 w = f[(size_t)k * V + s];
        p[2 * k] = mk(w.x, w.y);
        p[2 * k + 1] = mk(w.z, w.w);
    }
}
DDWC_HD void store_spinor(double2* __restrict__ f, int V, int s, const cx<double> p[12]) {
#pragma unroll
    for (int c = 0; c < 12; ++c) f[(size_t)c * V + s] = make_double2(p[c].re, p[c].im);
}
DDWC_HD void store_spinor(float4* __restrict__ f, int V, int s, const cx<float> p[12]) {
#pragma unroll
    for (int k = 0; k < 6; ++k)
        f[(size_t)k * V + s] = make_float4(p[2 * k].re, p[2 * k].im, p[2 * k + 1].re, p[2 * k + 1].im);
}

template <class R>
DDWC_HD void load_link(const cx<R>* __restrict__ U, int V, int mu, int s, cx<R> u[9]) {
    const cx<R>* base = U + (size_t)mu * 9 * V + s;
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = base[(size_t)k * V];
}

// The 36 reals of chiral block `blk` of the clover term at site s:
// d[0..5] = diagonal, o[0..29] = upper off-diagonal (re, im) in row order.
DDWC_HD void load_clover_block(const double2* __restrict__ K, int V, int s, int blk, double d[6],
                                                  double o[30]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double2 w = K[(size_t)(3 * blk + k) * V + s];
        d[2 * k] = w.x;
        d[2 * k + 1] = w.y;
    }
#pragma unroll
    for (int k = 0; k < 15; ++k) {
        double2 w = K[(size_t)(6 + 15 * blk + k) * V + s];
        o[2 * k] = w.x;
        o[2 * k + 1] = w.y;
    }
}
// FP32: reals 0..11 are words 0..2; block 0 off-diagonal reals 12..41 start in word 3,
// block 1 reals 42..71 start at word 10 offset 2.  Load the 9 words that cover a block.
DDWC_HD void load_clover_block(const float4* __restrict__ K, int V, int s, int blk, float d[6],
                                                  float o[30]) {
    float w[40];
    const int w0 = blk == 0 ? 3 : 10;  // first word holding off-diagonal reals of this block
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        float4 q = K[(size_t)(w0 + k) * V + s];
        w[4 * k] = q.x;
        w[4 * k + 1] = q.y;
        w[4 * k + 2] = q.z;
        w[4 * k + 3] = q.w;
    }
    const int sh = blk == 0 ? 0 : 2;  // reals 42.. start at offset 2 of word 10
#pragma unroll
    for (int k = 0; k < 30; ++k) o[k] = w[sh + k];
    // diagonal reals 6*blk .. 6*blk+5 live in words 0..2
    float4 q0 = K[(size_t)(blk == 0 ? 0 : 1) * V + s];
    float4 q1 = K[(size_t)(blk == 0 ? 1 : 2) * V + s];
    if (blk == 0) {
        d[0] = q0.x; d[1] = q0.y; d[2] = q0.z; d[3] = q0.w; d[4] = q1.x; d[5] = q1.y;
    } else {
        d[0] = q0.z; d[1] = q0.w; d[2] = q1.x; d[3] = q1.y; d[4] = q1.z; d[5] = q1.w;
    }
}

// Keeps the instruction scheduler from hoisting the next direction's loads above the
// current direction's arithmetic (which would hold all eight neighbours in registers).
DDWC_HD void sched_fence() {
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_sched_barrier(0);
#endif
}

// y = (4 + m) psi + C psi with the two packed Hermitian 6x6 blocks, one block at a time.
template <class R>
DDWC_HD void apply_diag(const typename Traits<R>::word* __restrict__ K, int V, int s, R mass4,
                                           const cx<R> p[12], cx<R> y[12]) {
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
        R d[6], o[30];
        load_clover_block(K, V, s, blk, d, o);
        const cx<R>* v = p + 6 * blk;
        cx<R>* w = y + 6 * blk;
#pragma unroll
        for (int i = 0; i < 6; ++i) w[i] = (mass4 + d[i]) * v[i];
        int k = 0;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
#pragma unroll
            for (int j = i + 1; j < 6; ++j) {
                cx<R> aij = mk(o[2 * k], o[2 * k + 1]);
                w[i] = w[i] + aij * v[j];
                w[j] = w[j] + conj_mul(aij, v[i]);
                ++k;
            }
        }
        sched_fence();
    }
}

// Spin structure of the hop terms in the chiral basis.  With q the neighbour spinor
// (spins 0..3), the projected half spinor of (1 - dir g_mu) q is
//     h0 = q0 + dir a0 q[i0],   h1 = q1 + dir a1 q[5 - i0],
// and after k = U h (forward) or U^+ h (backward) the four spins of the hop are
//     (k0, k1, dir b0 k[j0], dir b1 k[1 - j0]).
// a0, a1, b0, b1 are in {+-1, +-i}; the backward (1 + g_mu) terms only flip their sign.
struct HopSpin {
    int i0, j0;
    float a0r, a0i, a1r, a1i, b0r, b0i, b1r, b1i;
};

DDWC_HD HopSpin hop_spin(int mu) {
    HopSpin h;
    switch (mu) {
        case 0: h = HopSpin{2, 0, 1, 0, 1, 0, 1, 0, 1, 0}; break;     // h = q_u + q_l,          l = k
        case 1: h = HopSpin{3, 1, 0, 1, 0, 1, 0, -1, 0, -1}; break;   // h = q_u + i s1 q_l,     l = -i s1 k
        case 2: h = HopSpin{3, 1, 1, 0, -1, 0, -1, 0, 1, 0}; break;   // h = q_u + i s2 q_l,     l = -i s2 k
        default: h = HopSpin{2, 0, 0, 1, 0, -1, 0, -1, 0, 1}; break;  // h = q_u + i s3 q_l,     l = -i s3 k
    }
    return h;
}

template <class R>
DDWC_HD cx<R> cscale(float re, float im, cx<R> z) {
    return mk((R)re * z.re - (R)im * z.im, (R)re * z.im + (R)im * z.re);
}

// acc += fac * (1 - dir g_mu) W q, W = U (dir = +1) or U^+ (dir = -1).
template <class R>
DDWC_HD void hop_accumulate(int mu, int dir, const cx<R> u[9], const cx<R> q[12], R fac, cx<R> acc[12]) {
    const HopSpin hs = hop_spin(mu);
    const R sg = (R)dir;
    cx<R> h0[3], h1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cx<R> x0 = hs.i0 == 2 ? q[6 + a] : q[9 + a];
        const cx<R> x1 = hs.i0 == 2 ? q[9 + a] : q[6 + a];
        h0[a] = q[a] + sg * cscale(hs.a0r, hs.a0i, x0);
        h1[a] = q[3 + a] + sg * cscale(hs.a1r, hs.a1i, x1);
    }
    cx<R> w[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) w[3 * a + b] = dir > 0 ? u[3 * a + b] : mk(u[3 * b + a].re, -u[3 * b + a].im);
    cx<R> k0[3], k1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        k0[a] = fac * (w[3 * a] * h0[0] + w[3 * a + 1] * h0[1] + w[3 * a + 2] * h0[2]);
        k1[a] = fac * (w[3 * a] * h1[0] + w[3 * a + 1] * h1[1] + w[3 * a + 2] * h1[2]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        acc[a] = acc[a] + k0[a];
        acc[3 + a] = acc[3 + a] + k1[a];
        const cx<R> y0 = hs.j0 == 0 ? k0[a] : k1[a];
        const cx<R> y1 = hs.j0 == 0 ? k1[a] : k0[a];
        acc[6 + a] = acc[6 + a] + sg * cscale(hs.b0r, hs.b0i, y0);
        acc[9 + a] = acc[9 + a] + sg * cscale(hs.b1r, hs.b1i, y1);
    }
}

// Neighbour one step in direction dir (+1 / -1) along mu: index, same-block flag, and the
// time-boundary factor of the hop.
DDWC_HD int neighbour_rt(const Geom& g, int s, const Site& S, int mu, int dir, bool& inside, int& bc) {
    return dir > 0 ? neighbour<+1>(g, s, S, mu, inside, bc) : neighbour<-1>(g, s, S, mu, inside, bc);
}

// Which hops a site operator includes.
enum HopSet { HOPS_NONE = 0, HOPS_ALL = 1, HOPS_INSIDE = 2, HOPS_CROSSING = 3 };

// y = [diag] (4+m+C) psi(s) - 1/2 sum over the selected hops.  `in` points at one RHS.
// The diagonal part is applied first; the hops then accumulate into y with the factor
// -1/2 (times the time-boundary sign) folded into the half-spinor products.
template <class R, bool DIAG, int HOPS>
DDWC_HD void site_operator(const Geom& g, int s, const typename Traits<R>::word* __restrict__ in,
                                              const cx<R>* __restrict__ U, const typename Traits<R>::word* __restrict__ K,
                                              R mass4, cx<R> y[12]) {
    const int V = g.V;
    if (DIAG) {
        cx<R> c[12];
        load_spinor(in, V, s, c);
        apply_diag<R>(K, V, s, mass4, c, y);
        sched_fence();
    } else {
#pragma unroll
        for (int c = 0; c < 12; ++c) y[c] = mk(R(0), R(0));
    }
    if (HOPS != HOPS_NONE) {
        const Site S = decode(g, s);
        // one direction per trip: only one neighbour spinor and link are live at a time
#pragma unroll 1
        for (int d = 0; d < 8; ++d) {
            const int mu = d >> 1, dir = (d & 1) ? -1 : 1;
            bool inside;
            int bc;
            const int t = neighbour_rt(g, s, S, mu, dir, inside, bc);
            const bool take = HOPS == HOPS_ALL || (HOPS == HOPS_INSIDE && inside) || (HOPS == HOPS_CROSSING && !inside);
            if (take) {
                cx<R> q[12], u[9];
                load_spinor(in, V, t, q);
                load_link(U, V, mu, dir > 0 ? s : t, u);
                hop_accumulate<R>(mu, dir, u, q, R(-0.5) * R(bc), y);
            }
        }
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

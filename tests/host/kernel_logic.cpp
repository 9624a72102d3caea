// Host-side execution of the library's per-site device code (test harness only).
// The same __host__ __device__ functions the HIP kernels call (geometry, spin
// projection, clover packing and application) run here on the CPU over every site,
// so their logic can be compared with the FP64 oracle without a GPU.
#include <vector>

#include "../../paper_1211_1214_amd/csrc/clover_build.h"

using namespace ddwc;

// mode: 0 full operator, 1 Dirichlet blocks of colour `colour` (other colour zero),
//       2 hops crossing block faces into colour `colour` (other colour zero).
extern "C" int host_apply(const int* lat, const int* blk, int tbc, double csw, const double* links_canon,
                          const double* in_canon, double kappa, int mode, int colour, double* out_canon,
                          double* clover_out) {
    Geom g = make_geom(lat, blk, tbc);
    const int V = g.V;
    std::vector<cx<double>> U((size_t)36 * V);
    std::vector<int> can(V);
    for (int s = 0; s < V; ++s) {
        Site S = decode(g, s);
        can[s] = canonical_index(g, S);
        for (int mu = 0; mu < 4; ++mu)
            for (int k = 0; k < 9; ++k) {
                const double* src = links_canon + 2 * (((size_t)mu * V + can[s]) * 9 + k);
                U[((size_t)mu * 9 + k) * V + s] = mk(src[0], src[1]);
            }
    }
    std::vector<int> nbr((size_t)8 * V);
    for (int s = 0; s < V; ++s) {
        const Site S = decode(g, s);
        for (int mu = 0; mu < 4; ++mu) {
            nbr[(size_t)(2 * mu) * V + s] = table_entry<+1>(g, s, S, mu);
            nbr[(size_t)(2 * mu + 1) * V + s] = table_entry<-1>(g, s, S, mu);
        }
    }
    std::vector<double2> K((size_t)36 * V), in((size_t)12 * V);
    for (int s = 0; s < V; ++s) {
        double a[72];
        clover_site(g, U.data(), csw, s, a);
        for (int k = 0; k < 36; ++k) K[(size_t)k * V + s] = make_double2(a[2 * k], a[2 * k + 1]);
        if (clover_out)
            for (int k = 0; k < 72; ++k) clover_out[(size_t)can[s] * 72 + k] = a[k];
        for (int c = 0; c < 12; ++c) {
            const double* src = in_canon + 2 * ((size_t)can[s] * 12 + c);
            in[(size_t)c * V + s] = make_double2(src[0], src[1]);
        }
    }
    const double mass4 = 4.0 + (1.0 / (2.0 * kappa) - 4.0);
    for (int s = 0; s < V; ++s) {
        cx<double> y[12];
        const int c_s = s / (V / 2);
        if (mode == 0)
            site_operator<double, true, HOPS_ALL>(g, s, in.data(), U.data(), K.data(), nbr.data(), mass4, y, 8);
        else if (mode == 1 && c_s == colour)
            site_operator<double, true, HOPS_INSIDE>(g, s, in.data(), U.data(), K.data(), nbr.data(), mass4, y, 8);
        else if (mode == 2 && c_s == colour)
            site_operator<double, false, HOPS_CROSSING>(g, s, in.data(), U.data(), nullptr, nbr.data(), 0.0, y, 8);
        else
            for (int c = 0; c < 12; ++c) y[c] = mk(0.0, 0.0);
        for (int c = 0; c < 12; ++c) {
            out_canon[2 * ((size_t)can[s] * 12 + c)] = y[c].re;
            out_canon[2 * ((size_t)can[s] * 12 + c) + 1] = y[c].im;
        }
    }
    return 0;
}

// Even-odd operator on the host with the library's own helpers: y_e = Mee x_e with
// Mee = A_ee - 1/4 H_eo A_oo^-1 H_oe, half fields built as the setup kernel builds them.
// Output in canonical layout, zero on odd sites.  Requires every block extent even.
#include "../../paper_1211_1214_amd/csrc/eo.h"
extern "C" int host_eo_apply(const int* lat, const int* blk, int tbc, double csw, const double* links_canon,
                             const double* in_canon, double kappa, double* out_canon) {
    Geom g = make_geom(lat, blk, tbc);
    if (!g.eo) return -1;
    const int V = g.V, n2 = V / 2;
    std::vector<cx<double>> U((size_t)36 * V);
    std::vector<int> can(V), nbr((size_t)8 * V);
    for (int s = 0; s < V; ++s) {
        const Site S = decode(g, s);
        can[s] = canonical_index(g, S);
        for (int mu = 0; mu < 4; ++mu) {
            for (int k = 0; k < 9; ++k) {
                const double* src = links_canon + 2 * (((size_t)mu * V + can[s]) * 9 + k);
                U[((size_t)mu * 9 + k) * V + s] = mk(src[0], src[1]);
            }
            nbr[(size_t)(2 * mu) * V + s] = table_entry<+1>(g, s, S, mu);
            nbr[(size_t)(2 * mu + 1) * V + s] = table_entry<-1>(g, s, S, mu);
        }
    }
    const double mass4 = 4.0 + (1.0 / (2.0 * kappa) - 4.0);
    std::vector<cx<double>> Uh((size_t)2 * 36 * n2);
    std::vector<double2> Kh((size_t)2 * 36 * n2), Ah((size_t)36 * n2), xe((size_t)12 * n2), xo((size_t)12 * n2, make_double2(0, 0));
    std::vector<int> nh((size_t)2 * 8 * n2);
    for (int s = 0; s < V; ++s) {
        int p;
        const unsigned i = half_index(g, s, p);
        if (full_index(g, i, p) != (unsigned)s) return -2;
        for (int mu = 0; mu < 4; ++mu)
            for (int k = 0; k < 9; ++k) Uh[(((size_t)p * 4 + mu) * 9 + k) * n2 + i] = U[((size_t)mu * 9 + k) * V + s];
        double a[72], b[72];
        clover_site(g, U.data(), csw, s, a);
        for (int k = 0; k < 36; ++k) Kh[((size_t)p * 36 + k) * n2 + i] = make_double2(a[2 * k], a[2 * k + 1]);
        if (p == 1) {
            clover_inverse_site(a, mass4, b);
            for (int k = 0; k < 36; ++k) Ah[(size_t)k * n2 + i] = make_double2(b[2 * k], b[2 * k + 1]);
        }
        for (int d = 0; d < 8; ++d) nh[((size_t)p * 8 + d) * n2 + i] = half_entry(g, nbr[(size_t)d * V + s]);
        if (p == 0)
            for (int c = 0; c < 12; ++c) {
                const double* src = in_canon + 2 * ((size_t)can[s] * 12 + c);
                xe[(size_t)c * n2 + i] = make_double2(src[0], src[1]);
            }
    }
    const cx<double>* U0 = Uh.data();
    const cx<double>* U1 = Uh.data() + (size_t)36 * n2;
    // t_o = A_oo^-1 H_oe x_e
    for (int i = 0; i < n2; ++i) {
        cx<double> acc[12], w[12];
        hop_sum<double, HOPS_ALL, false>(n2, i, xe.data(), U1, U0, nh.data() + (size_t)8 * n2, acc, 8);
        for (int c = 0; c < 12; ++c) w[c] = mk(0.0, 0.0);
        apply_diag<double>(Ah.data(), n2, i, 0.0, acc, w, 0.0);
        store_spinor(xo.data(), n2, i, w);
    }
    for (size_t k = 0; k < (size_t)24 * V; ++k) out_canon[k] = 0;
    // y_e = A_ee x_e - 1/4 H_eo t_o
    for (int i = 0; i < n2; ++i) {
        cx<double> acc[12], c[12];
        hop_sum<double, HOPS_ALL, false>(n2, i, xo.data(), U0, U1, nh.data(), acc, 8);
        load_spinor(xe.data(), n2, i, c);
        apply_diag<double>(Kh.data(), n2, i, mass4, c, acc, -0.25);
        const int s = can[full_index(g, i, 0)];
        for (int k = 0; k < 12; ++k) {
            out_canon[2 * ((size_t)s * 12 + k)] = acc[k].re;
            out_canon[2 * ((size_t)s * 12 + k) + 1] = acc[k].im;
        }
    }
    return 0;
}

// Link gradient of Re <a, D(U) b> (one RHS, weight 1) with the library's force code: hop part
// and clover part, in canonical layout [4][V][3][3] (re, im).
#include "../../paper_1211_1214_amd/csrc/force.h"
struct HostAdder {
    std::vector<cx<double>>* G;
    int V;
    void operator()(int mu, int s, const M3& m) const {
        for (int k = 0; k < 9; ++k) (*G)[((size_t)mu * 9 + k) * V + s] = (*G)[((size_t)mu * 9 + k) * V + s] + m.a[k];
    }
};
extern "C" int host_force(const int* lat, const int* blk, int tbc, double csw, const double* links_canon,
                          const double* a_canon, const double* b_canon, double* grad_canon) {
    Geom g = make_geom(lat, blk, tbc);
    const int V = g.V;
    std::vector<cx<double>> U((size_t)36 * V), G((size_t)36 * V, mk(0.0, 0.0));
    std::vector<int> can(V), nbr((size_t)8 * V);
    std::vector<double2> a((size_t)12 * V), b((size_t)12 * V);
    for (int s = 0; s < V; ++s) {
        const Site S = decode(g, s);
        can[s] = canonical_index(g, S);
        for (int mu = 0; mu < 4; ++mu) {
            for (int k = 0; k < 9; ++k) {
                const double* src = links_canon + 2 * (((size_t)mu * V + can[s]) * 9 + k);
                U[((size_t)mu * 9 + k) * V + s] = mk(src[0], src[1]);
            }
            nbr[(size_t)(2 * mu) * V + s] = table_entry<+1>(g, s, S, mu);
            nbr[(size_t)(2 * mu + 1) * V + s] = table_entry<-1>(g, s, S, mu);
        }
        for (int c = 0; c < 12; ++c) {
            a[(size_t)c * V + s] = make_double2(a_canon[2 * ((size_t)can[s] * 12 + c)], a_canon[2 * ((size_t)can[s] * 12 + c) + 1]);
            b[(size_t)c * V + s] = make_double2(b_canon[2 * ((size_t)can[s] * 12 + c)], b_canon[2 * ((size_t)can[s] * 12 + c) + 1]);
        }
    }
    const double w = 1.0;
    for (int s = 0; s < V; ++s)
        for (int mu = 0; mu < 4; ++mu) force_hop_site(g, nbr.data(), a.data(), b.data(), &w, 1, G.data(), s, mu);
    if (csw != 0.0) {
        HostAdder add{&G, V};
        for (int y = 0; y < V; ++y) force_clover_site(g, U.data(), csw, a.data(), b.data(), &w, 1, y, add);
    }
    for (int s = 0; s < V; ++s)
        for (int mu = 0; mu < 4; ++mu)
            for (int k = 0; k < 9; ++k) {
                const cx<double> v = G[((size_t)mu * 9 + k) * V + s];
                grad_canon[2 * (((size_t)mu * V + can[s]) * 9 + k)] = v.re;
                grad_canon[2 * (((size_t)mu * V + can[s]) * 9 + k) + 1] = v.im;
            }
    return 0;
}

// FP16 spinor storage: store then load one spinor (24 reals) through the library's code.
extern "C" int host_h16_roundtrip(const double* in, double* out, float* scale_out) {
    struct alignas(16) Buf {
        hw16 w[3];
        float scale[4];
    } buf;
    cx<float> p[12], q[12];
    for (int c = 0; c < 12; ++c) p[c] = mk((float)in[2 * c], (float)in[2 * c + 1]);
    store_spinor(buf.w, 1, 0, p);
    load_spinor((const hw16*)buf.w, 1, 0, q);
    for (int c = 0; c < 12; ++c) {
        out[2 * c] = q[c].re;
        out[2 * c + 1] = q[c].im;
    }
    *scale_out = buf.scale[0];
    return 0;
}

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

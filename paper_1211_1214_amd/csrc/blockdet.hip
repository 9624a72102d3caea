// Exact log-determinants of the Dirichlet Schwarz blocks D_k (the block factor of Eq. 7).
//
// With every block extent even, the odd sites of a block are eliminated first (eo.h):
//     det D_k = prod_{x odd in k} det A(x) * det M_k,   M_k = A_ee - 1/4 H^k_eo A_oo^-1 H^k_oe,
// so the dense matrix is 12 Vb/2 square.  A(x) = (4 + m) + C(x) is a pair of Hermitian
// positive definite 6x6 blocks (ln det by Cholesky).  Otherwise D_k itself (12 Vb square) is
// assembled.  One thread builds one column of one block's matrix from the library's own
// site operators (column-major, as the LU expects); a batched complex LU with partial
// pivoting (rocSOLVER getrf) factors the batch, and ln|det| = sum ln|U_ii| with the sign
// from the diagonal phases and the row interchanges.  det D_k is real by gamma_5-hermiticity.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "ddwc_internal.h"
#include "eo.h"

namespace ddwc {

__device__ void packed_at(const double2* __restrict__ K, unsigned V, unsigned s, double a[72]) {
    for (int k = 0; k < 36; ++k) {
        const double2 w = K[(size_t)k * V + s];
        a[2 * k] = w.x;
        a[2 * k + 1] = w.y;
    }
}

// contribution of the unit spinor v at site `from` to (H v)(to) through the hop of `to` in
// direction dp (whose neighbour is `from`), added to acc
__device__ void hop_from(const Geom& g, const cx<double>* __restrict__ U, int dp, unsigned to, unsigned from,
                         const cx<double> v[12], cx<double> acc[12]) {
    cx<double> u[9];
    load_link(U, g.V, dp >> 1, (dp & 1) ? from : to, u);
    hop_dispatch<double>(dp, u, v, acc);
}

// Columns of M_k (even-odd) for blocks r0 .. r0 + nb - 1 of `colour`.
__global__ void k_bd_assemble_eo(Geom g, const cx<double>* __restrict__ U, const double2* __restrict__ K,
                                 const int* __restrict__ nbr, double mass4, int colour, int r0, int nb,
                                 cx<double>* __restrict__ Mat) {
    const int n = 12 * g.hvb;
    const long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= (long)nb * n) return;
    const int bi = (int)(j / n), col = (int)(j - (long)bi * n);
    const int B = colour * g.NBc + r0 + bi;
    const unsigned base = (unsigned)B * g.Vb;
    const int h0 = col / 12, c0 = col - 12 * h0;
    const unsigned e0 = base + h0;  // even sites come first in a block
    cx<double>* M = Mat + (size_t)bi * n * n + (size_t)col * n;
    cx<double> v[12], y[12], w[12], z[12];
    for (int c = 0; c < 12; ++c) v[c] = mk(0.0, 0.0);
    v[c0] = mk(1.0, 0.0);
    double a[72], ai[72];
    packed_at(K, g.V, e0, a);
    packed_apply(a, mass4, v, y);
    for (int r = 0; r < 12; ++r) M[12 * h0 + r] = M[12 * h0 + r] + y[r];
    for (int d = 0; d < 8; ++d) {
        const int e = nbr[(size_t)d * g.V + e0];
        const unsigned t = e < 0 ? (unsigned)~e : (unsigned)e;
        if (t / (unsigned)g.Vb != (unsigned)B) continue;  // Dirichlet: hops inside the block only
        for (int c = 0; c < 12; ++c) w[c] = mk(0.0, 0.0);
        hop_from(g, U, d ^ 1, t, e0, v, w);  // (H_oe v)(t)
        packed_at(K, g.V, t, a);
        clover_inverse_site(a, mass4, ai);
        packed_apply(ai, 0.0, w, y);  // A_oo^-1 at t
        for (int d2 = 0; d2 < 8; ++d2) {
            const int e2 = nbr[(size_t)d2 * g.V + t];
            const unsigned i = e2 < 0 ? (unsigned)~e2 : (unsigned)e2;
            if (i / (unsigned)g.Vb != (unsigned)B) continue;
            for (int c = 0; c < 12; ++c) z[c] = mk(0.0, 0.0);
            hop_from(g, U, d2 ^ 1, i, t, y, z);  // (H_eo y)(i)
            const unsigned hi = i - base;
            for (int r = 0; r < 12; ++r) M[12 * hi + r] = M[12 * hi + r] - 0.25 * z[r];
        }
    }
}

// Columns of D_k itself (any block shape).
__global__ void k_bd_assemble_full(Geom g, const cx<double>* __restrict__ U, const double2* __restrict__ K,
                                   const int* __restrict__ nbr, double mass4, int colour, int r0, int nb,
                                   cx<double>* __restrict__ Mat) {
    const int n = 12 * g.Vb;
    const long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= (long)nb * n) return;
    const int bi = (int)(j / n), col = (int)(j - (long)bi * n);
    const int B = colour * g.NBc + r0 + bi;
    const unsigned base = (unsigned)B * g.Vb;
    const int l0 = col / 12, c0 = col - 12 * l0;
    const unsigned x0 = base + l0;
    cx<double>* M = Mat + (size_t)bi * n * n + (size_t)col * n;
    cx<double> v[12], y[12];
    for (int c = 0; c < 12; ++c) v[c] = mk(0.0, 0.0);
    v[c0] = mk(1.0, 0.0);
    double a[72];
    packed_at(K, g.V, x0, a);
    packed_apply(a, mass4, v, y);
    for (int r = 0; r < 12; ++r) M[12 * l0 + r] = M[12 * l0 + r] + y[r];
    for (int d = 0; d < 8; ++d) {
        const int e = nbr[(size_t)d * g.V + x0];
        const unsigned t = e < 0 ? (unsigned)~e : (unsigned)e;
        if (t / (unsigned)g.Vb != (unsigned)B) continue;
        for (int c = 0; c < 12; ++c) y[c] = mk(0.0, 0.0);
        hop_from(g, U, d ^ 1, t, x0, v, y);
        const unsigned lt = t - base;
        for (int r = 0; r < 12; ++r) M[12 * lt + r] = M[12 * lt + r] - 0.5 * y[r];
    }
}

// sum over the odd sites of each block of `colour` of ln det A(x), one workgroup per block
__global__ void k_bd_oddlogdet(Geom g, const double2* __restrict__ K, double mass4, int colour, double* out) {
    __shared__ double lds[16];
    const int B = colour * g.NBc + blockIdx.x;
    double v[1] = {0};
    for (int l = g.hvb + threadIdx.x; l < g.Vb; l += blockDim.x) {
        double a[72];
        packed_at(K, g.V, (unsigned)B * g.Vb + l, a);
        v[0] += herm6_logdet(a, a + 12, mass4) + herm6_logdet(a + 6, a + 42, mass4);
    }
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = v[0];
}

// ln|det| and the phase of det from the LU factors of one matrix per workgroup:
// out[2 b] = sum ln|U_ii|, out[2 b + 1] = sum arg U_ii + pi * (number of row interchanges).
__global__ void k_bd_lu_logdet(int n, const cx<double>* __restrict__ Mat, const int* __restrict__ ipiv,
                               double* out) {
    __shared__ double lds[2 * 16];
    const cx<double>* M = Mat + (size_t)blockIdx.x * n * n;
    const int* piv = ipiv + (size_t)blockIdx.x * n;
    double v[2] = {0, 0};
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const cx<double> d = M[(size_t)i * n + i];
        v[0] += 0.5 * log(d.re * d.re + d.im * d.im);
        v[1] += atan2(d.im, d.re) + (piv[i] != i + 1 ? M_PI : 0.0);
    }
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = v[0];
        out[2 * blockIdx.x + 1] = v[1];
    }
}

int block_logdet_run(Exec& e, const Geom& g, const cx<double>* U, const double2* K, const int* nbr, double mass4,
                     int colour, int r0, int nb, void* rb, cx<double>* Mat, int* ipiv, int* info, double* lu_out) {
    const bool eo = g.eo != 0;
    const int n = eo ? 12 * g.hvb : 12 * g.Vb;
    {
        Timed t(e, 4, 0);
        if (hipMemsetAsync(Mat, 0, (size_t)nb * n * n * sizeof(cx<double>), e.stream) != hipSuccess) return -1;
        const long nt = (long)nb * n;
        const int grid = (int)((nt + 127) / 128);
        if (eo)
            k_bd_assemble_eo<<<grid, 128, 0, e.stream>>>(g, U, K, nbr, mass4, colour, r0, nb, Mat);
        else
            k_bd_assemble_full<<<grid, 128, 0, e.stream>>>(g, U, K, nbr, mass4, colour, r0, nb, Mat);
    }
    rocblas_handle h = (rocblas_handle)rb;
    if (rocblas_set_stream(h, e.stream) != rocblas_status_success) return -2;
    {
        Timed t(e, 4, 0);
        if (rocsolver_zgetrf_strided_batched(h, n, n, (rocblas_double_complex*)Mat, n, (rocblas_stride)n * n, ipiv,
                                             n, info, nb) != rocblas_status_success)
            return -3;
    }
    {
        Timed t(e, 4, 0);
        k_bd_lu_logdet<<<nb, 256, 0, e.stream>>>(n, Mat, ipiv, lu_out);
    }
    return 0;
}

void launch_bd_oddlogdet(Exec& e, const Geom& g, const double2* K, double mass4, int colour, double* out) {
    Timed t(e, 4, 0);
    k_bd_oddlogdet<<<g.NBc, 256, 0, e.stream>>>(g, K, mass4, colour, out);
}

void* blas_handle_create() {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) return nullptr;
    return (void*)h;
}
void blas_handle_destroy(void* h) {
    if (h) rocblas_destroy_handle((rocblas_handle)h);
}

}  // namespace ddwc

// Host-side declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <vector>

#include "ddwc_device.h"

namespace ddwc {

// Per-RHS BiCGStab scalars, kept on the device so that iterations need no host round trip.
struct BiState {
    double rho[2], alpha[2], omega[2], beta[2];
    double rr;    // ||r||^2 after the last iteration
    double thr2;  // stop when rr <= thr2
    int active;   // 0 once converged (or broken down): updates become no-ops
    int broken;   // breakdown (zero denominator) detected
};

// Stages of the global BiCGStab's finalize (k_finalize): ST_OMEGA takes (t, s), (t, t), (rh, s) and
// (rh, t) and sets omega, the next rho = (rh, s) - omega (rh, t) = (rh, r_new) and beta, so that one
// kernel updates x, r and p; ST_RR takes ||r_new||^2 and decides convergence.
enum Stage { ST_SUM = 0, ST_INIT = 1, ST_ALPHA = 2, ST_OMEGA = 3, ST_RR = 4 };

// Spinor masks for import / combination kernels.
enum Mask { MASK_ALL = 0, MASK_P = 1, MASK_BLACK = 2, MASK_WHITE = 3 };

// Kernel timing with HIP events (measurement only).
struct Profiler {
    bool on = false;
    struct Pair {
        hipEvent_t a, b;
        int kclass;
        double bytes;
    };
    std::vector<Pair> pending;
    std::vector<hipEvent_t> pool;
    long long launches[8] = {0};
    double ms[8] = {0};
    double bytes[8] = {0};
    hipEvent_t get();
    void begin(hipStream_t s, int kclass, double bytes, Pair& p);
    void end(hipStream_t s, Pair& p);
    void harvest();  // synchronises on the pending events
    void reset();
    ~Profiler();
};

struct Exec {
    hipStream_t stream;
    Profiler* prof;
    const int* nbr;        // neighbour table [8][V] of the context
    int blk_threads = 0;   // workgroup size of the block-solver kernels (0: the default rule)
    int blk_lds = 0;       // KiB of LDS reserved per persistent block-solver workgroup (caps residency)
};

// RAII-free scoped timing helper used by the launchers.
struct Timed {
    Exec& e;
    Profiler::Pair p;
    bool active;
    Timed(Exec& ex, int kclass, double bytes) : e(ex), active(ex.prof && ex.prof->on) {
        if (active) e.prof->begin(e.stream, kclass, bytes, p);
    }
    ~Timed() {
        if (active) e.prof->end(e.stream, p);
    }
};

// ------------------------------------------------------------------ launchers (kernels.hip)
constexpr int WG = 256;  // sites per workgroup of the site-parallel kernels
constexpr int NPART = 8; // doubles per partial-sum slot

inline int tiles_of(int n) { return (n + WG - 1) / WG; }

// Links to the internal layouts: U64, U32 entry-major [4][9][V].
void launch_links_import(Exec& e, const Geom& g, const void* canon, cx<double>* U64, cx<float>* U32);
// Own-site link records [n][8][9] (LK_OWN) of n sites from entry-major forward links Uf ([4][9][n])
// and Ub (the neighbours', [4][9][n]) and the table nbr [8][n].
void launch_links_own(Exec& e, unsigned n, const cx<float>* Uf, const cx<float>* Ub, const int* nbr,
                      cx<float>* Lown);
// Full-lattice FP32 Dslash on RHS-innermost fields [6][V][nrhs] (canonical FP64 in and out), with
// the own-site link records Us [V][8][9]; op_threads (128, 256 or 512; 256 below nrhs) threads per
// workgroup, tiles dispatched in `order` (null: index order; dslash_ri32_tiles() entries).
void launch_import_ri32(Exec& e, const Geom& g, const void* canon, float4* out, int nrhs);
void launch_export_ri32(Exec& e, const Geom& g, const float4* in, void* canon, int nrhs);
void launch_dslash_ri32(Exec& e, const Geom& g, const cx<float>* Us, const float4* K, double mass4, const float4* in,
                        float4* out, int nrhs, int kclass, double bytes, int op_threads = WG,
                        const int* order = nullptr);
int dslash_ri32_tiles(const Geom& g, int nrhs, int op_threads);
void launch_nbr_build(Exec& e, const Geom& g, int* nbr);
void launch_clover_build(Exec& e, const Geom& g, const cx<double>* U64, double csw, double2* K64, float4* K32);

template <class R>
void launch_import(Exec& e, const Geom& g, const void* canon, typename Traits<R>::word* out, int nrhs, int mask);
template <class R>
void launch_export(Exec& e, const Geom& g, const typename Traits<R>::word* in, void* canon, int nrhs, int mask);

// out = D(m) in over all sites (no reductions).
template <class R>
void launch_dslash(Exec& e, const Geom& g, const cx<R>* U, const typename Traits<R>::word* K, double mass4,
                   const typename Traits<R>::word* in, typename Traits<R>::word* out, int nrhs, int kclass,
                   double bytes);
// out = D(m) in, partial[rhs][tile] = (w, out) (complex).
template <class R>
void launch_dslash_dot(Exec& e, const Geom& g, const cx<R>* U, const typename Traits<R>::word* K, double mass4,
                       const typename Traits<R>::word* in, typename Traits<R>::word* out,
                       const typename Traits<R>::word* w, double* part, int nrhs, int kclass, double bytes);
// out = D(m) in, partials (out, in) complex, (out, out), (rh, in) and (rh, out) complex.
template <class R>
void launch_dslash_dot4(Exec& e, const Geom& g, const cx<R>* U, const typename Traits<R>::word* K, double mass4,
                        const typename Traits<R>::word* in, typename Traits<R>::word* out,
                        const typename Traits<R>::word* rh, double* part, int nrhs, int kclass, double bytes);
// r = b - D(m) x, partial ||r||^2.
template <class R>
void launch_residual(Exec& e, const Geom& g, const cx<R>* U, const typename Traits<R>::word* K, double mass4,
                     const typename Traits<R>::word* x, const typename Traits<R>::word* b,
                     typename Traits<R>::word* r, double* part, int nrhs, int kclass, double bytes);
// Extents of an outer block decomposition (nested domain decomposition).
struct Ext4 {
    int v[4];
};

// out = hops crossing block faces into sites of colour `to_colour` (D_wb for white, D_bw for
// black); out is zero on the other colour (left untouched there with clear_other false, for
// consumers that read only colour to_colour: the block solves of that colour).  With cut, out is
// also zero outside the outer blocks (extents *cut) of colour cut_colour: the hops of the
// Dirichlet operator of those blocks.
template <class R>
void launch_hop(Exec& e, const Geom& g, const cx<R>* U, const typename Traits<R>::word* in,
                typename Traits<R>::word* out, int nrhs, int to_colour, const Ext4* cut = nullptr,
                int cut_colour = -1, bool clear_other = true);

// BiCGStab vector kernels on fields of n sites, nrhs RHS, per-RHS scalars in st, storage S
// (double, float or H16; H16 fields must be RHS-innermost).  ri selects the RHS-innermost
// layout [NCW][n][nrhs] (else [nrhs][NCW][n]); FP64 fields (r64, x64) are always RHS-major.
// Partial sums use vector_tiles() tiles per RHS.
int vector_tiles(unsigned n, int nrhs, bool ri);
template <class S>
void launch_bicg_init(Exec& e, unsigned n, bool ri, const double2* r64, const double* scale,
                      typename Traits<S>::word* r, typename Traits<S>::word* rh, typename Traits<S>::word* p,
                      typename Traits<typename Traits<S>::xs>::word* x, double* part, int nrhs);
template <class S>
void launch_bicg_s(Exec& e, unsigned n, bool ri, const BiState* st, const typename Traits<S>::word* r,
                   const typename Traits<S>::word* v, typename Traits<S>::word* s, int nrhs);
// x += alpha p + omega s; r = s - omega t; p = r + beta (p - omega v); partial ||r||^2.
template <class S>
void launch_bicg_xrp(Exec& e, unsigned n, bool ri, const BiState* st, typename Traits<typename Traits<S>::xs>::word* x,
                     typename Traits<S>::word* p, const typename Traits<S>::word* s, const typename Traits<S>::word* t,
                     const typename Traits<S>::word* v, typename Traits<S>::word* r, double* part, int nrhs);
// x64 += (1/scale) * x per RHS (RHS with scale 0 untouched); x in Traits<S>::xs.
template <class S>
void launch_accumulate(Exec& e, unsigned n, bool ri, const typename Traits<typename Traits<S>::xs>::word* x,
                       const double* scale, double2* x64, int nrhs);

// Sums partials per RHS in a fixed order and applies the BiCGStab stage update.
void launch_finalize(Exec& e, const double* part, int ntiles, int nrhs, double* sums, BiState* st, int stage,
                     const double* thr_rel2, int nv = -1);

// dst = src over n 16-byte words (streaming reference kernel).
void launch_stream_copy(Exec& e, const float4* src, float4* dst, size_t n);

// n double2 words of reproducible values in [-1/2, 1/2) (autotuner inputs).
void launch_fill_hash(Exec& e, double2* v, size_t n, uint64_t seed);

// FP64 helpers on internal vectors.
// z = a*x + b*y on sites selected by mask (others of z set to zero); x or y may be null (= 0).
void launch_axpby(Exec& e, const Geom& g, double a, const double2* x, double b, const double2* y, double2* z,
                  int nrhs, int mask);
// y += c_r x per RHS (c device, nrhs complex).
void launch_caxpy(Exec& e, const Geom& g, const double2* c, const double2* x, double2* y, int nrhs);
// nested domain decomposition: cut to the outer blocks of one colour, copy between two block layouts
void launch_region(Exec& e, const Geom& g, const Ext4& Bo, int colour, double2* v, int nrhs);
void launch_relayout(Exec& e, const Geom& gs, const Geom& gd, const double2* src, double2* dst, int nrhs);
constexpr int FP_BLOCKS = 1024;  // workgroups of the link fingerprint
void launch_link_fp(Exec& e, const void* links, size_t n, double* part);
// partials: (x, y) complex and (y, y) per RHS; x may equal y.
void launch_dots(Exec& e, const Geom& g, const double2* x, const double2* y, double* part, int nrhs);

// ------------------------------------------------------------------ derivatives (grad.hip)
// v <- gamma_5 v (negates spins 2, 3), in place, FP64 internal fields.
void launch_gamma5(Exec& e, const Geom& g, double2* v, int nrhs);
// G += d/dU sum_r w_r Re <a_r, D b_r>: the hop part (force_hop) and the clover part
// (force_clover, atomic adds).  G internal [4][9][V]; w device array [nrhs].
void launch_force_hop(Exec& e, const Geom& g, const int* nbr, const double2* a, const double2* b, const double* w,
                      int nrhs, cx<double>* G);
void launch_force_clover(Exec& e, const Geom& g, const cx<double>* U, double csw, const double2* a, const double2* b,
                         const double* w, int nrhs, cx<double>* G);
// internal link-shaped field -> canonical [4][V][3][3] complex128
void launch_links_export(Exec& e, const Geom& g, const cx<double>* G, void* canon);

// ------------------------------------------------------------------ block determinants (blockdet.hip)
// Assembles the dense block matrices (M_k when g.eo, else D_k) of blocks r0 .. r0 + nb - 1 of
// `colour` into Mat (column-major, nb x n x n), factors them (batched LU, handle rb) and
// writes per block (sum ln|U_ii|, phase) to lu_out[2 nb].  Returns 0 or a negative code.
int block_logdet_run(Exec& e, const Geom& g, const cx<double>* U, const double2* K, const int* nbr, double mass4,
                     int colour, int r0, int nb, void* rb, cx<double>* Mat, int* ipiv, int* info, double* lu_out);
// per block of `colour`: sum over its odd sites of ln det A(x)
void launch_bd_oddlogdet(Exec& e, const Geom& g, const double2* K, double mass4, int colour, double* out);
void* blas_handle_create();
void blas_handle_destroy(void* h);

// ------------------------------------------------------------------ even-odd (eo.hip)
// Half-field data of one precision: links, clover and neighbour table of each parity.
template <class R>
struct EoFields {
    unsigned n2;                                        // V / 2
    const cx<typename Traits<R>::link>* U[2];           // [4][9][n2] links of the sites of parity p
    const typename Traits<R>::kword* K[2];              // clover of the sites of parity p
    const int* nbr[2];                                  // [8][n2] neighbour half indices (other parity)
    int op_threads = WG;                                // workgroup size of the RHS-innermost operator kernels
    const int* order = nullptr;                         // their tile dispatch order (null: index order)
};

// Workgroup size and tile count of the operator kernels (launch_eo_hopinv / launch_eo_diaghop) on
// nrhs RHS: the RHS-innermost FP32 and FP16 kernels take op_threads (WG where it is below nrhs: a
// workgroup's partial sums need every RHS in it), the others WG (RHS-major: per tile of sites).
template <class R>
inline int eo_op_threads(const EoFields<R>& F, int nrhs, bool ri) {
    return ri && !std::is_same<R, double>::value && nrhs <= F.op_threads ? F.op_threads : WG;
}
template <class R>
inline int eo_op_tiles(const EoFields<R>& F, int nrhs, bool ri) {
    const long long n = ri ? (long long)F.n2 * nrhs : (long long)F.n2;
    const int t = eo_op_threads(F, nrhs, ri);
    return (int)((n + t - 1) / t);
}

// FP16 copy of n FP32 complex link entries.
void launch_links_to_half(Exec& e, size_t n, const cx<float>* src, cx<f16>* dst);
// Half-field links: entry-major Uh64, Uh32 [2][4][9][V/2].
void launch_eo_setup(Exec& e, const Geom& g, const cx<double>* U64, const double2* K64, const int* nbr,
                     cx<double>* Uh64, cx<float>* Uh32, double2* Kh64, float4* Kh32, int* nbr_eo);
// Own-site link records [2][V/2][8][9] (LK_OWN) read by the RHS-innermost kernels of the global
// solver, from Uh32 and the half-field neighbour tables.
void launch_eo_links_own(Exec& e, unsigned n2, const cx<float>* Uh32, const int* nbr_eo, cx<float>* Lown);
void launch_eo_inverse(Exec& e, unsigned V2, const double2* Kp, double mass4, double2* A64, float4* A32);
void launch_eo_split(Exec& e, const Geom& g, const double2* full, double2* he, double2* ho, int nrhs);
void launch_eo_merge(Exec& e, const Geom& g, const double2* he, const double2* ho, double2* full, int nrhs,
                     const double2* ho2 = nullptr, double w2 = 0.0);
// y_p = Ainv (c + alpha H_{p,1-p} x); c may be null, alpha = 0 skips the hops.  ri: the fields
// are RHS-innermost (as for the vector kernels).
template <class S>
void launch_eo_hopinv(Exec& e, const EoFields<S>& F, int p, bool ri, const typename Traits<S>::word* x,
                      const typename Traits<S>::word* c, double alpha, const typename Traits<S>::kword* Ainv,
                      typename Traits<S>::word* y, int nrhs, int kclass, double bytes);
// y_p = [A_pp] c + beta H_{p,1-p} t with epilogue epi (0 none, 1 dot(aux, y), 2 dots (y, c), (y, y),
// 3 residual y = aux - y with ||y||^2).
template <class S>
void launch_eo_diaghop(Exec& e, const EoFields<S>& F, int p, bool ri, int epi, bool use_a,
                       const typename Traits<S>::word* c, const typename Traits<S>::word* tv, double beta,
                       double mass4, const typename Traits<S>::word* aux, typename Traits<S>::word* y, double* part,
                       int nrhs, int kclass, double bytes);

// ------------------------------------------------------------------ even-odd block solver (block_eo.hip)
void launch_blk_prep(Exec& e, const Geom& g, const EoFields<double>& F, const double2* Ainv, const double2* b,
                     double2* bpe, double2* re, double2* xe, double2* to, double* bb, double* rr, int colour, int nrhs);
void launch_blk_resid(Exec& e, const Geom& g, const EoFields<double>& F, const double2* Ainv, const double2* bpe,
                      const double2* xe, double2* re, double2* to, double* rr, double mass4, int colour, int nrhs);
void launch_blk_recon(Exec& e, const Geom& g, const double2* to, const double2* th, const double2* xe, double2* x,
                      int colour, int nrhs);
template <class S>
void launch_blk_inner(Exec& e, const Geom& g, const EoFields<S>& F, const typename Traits<S>::kword* Ainv,
                      const double2* re, double2* xe, void* const w[7], const double* bb, const double* rr,
                      double mass4, double tol, int maxit, int* iters, int colour, int nrhs);
// The LDS-resident FP32 inner solver (both staged block fields in LDS, per-site iterates in
// registers): whether it takes this geometry with lds_max_bytes of LDS per workgroup, and its
// launch (slabs w[1], w[3], w[5] hold rh, v and the correction in FP32).
bool blk_lds_fits(const Geom& g, int lds_max_bytes);
void launch_blk_lds(Exec& e, const Geom& g, const EoFields<float>& F, const float4* Ainv, const double2* re,
                    double2* xe, void* const w[7], const double* bb, const double* rr, double mass4, double tol,
                    int maxit, int* iters, int colour, int nrhs);
// bytes of one RHS of a block-solver vector in the storage of precision `prec` (n2 = V/2)
size_t blk_slab_bytes(int prec, unsigned n2);

// ------------------------------------------------------------------ block solver (block_solver.hip)
struct BlockSolveArgs {
    const double2* b;     // FP64 right-hand sides, internal layout
    double2* x;           // FP64 solutions
    double2* r64;         // FP64 residual scratch
    void* w[6];           // inner-precision scratch vectors: r, rh, p, v, t, e
    int colour;
    int nrhs;
    double mass4;
    double tol;
    int maxit;
    int* iters;           // [nrhs][NBc] inner iterations per block
    int* outer;           // [nrhs][NBc] defect-correction steps per block
    double* relres;       // [nrhs][NBc] final FP64 relative residual per block
};
void launch_block_solve64(Exec& e, const Geom& g, const cx<double>* U, const double2* K, const BlockSolveArgs& a);
void launch_block_solve32(Exec& e, const Geom& g, const cx<double>* U64, const double2* K64, const cx<float>* U32,
                          const float4* K32, const BlockSolveArgs& a);
int block_solver_threads(const Geom& g);

}  // namespace ddwc

/*
 * ddwc — Schwarz-factorised stochastic determinant ratios for Wilson-clover
 * fermions on AMD Instinct MI355X (gfx950).  C ABI.
 *
 * The method: the Dirac operator in black/white Schwarz block form
 * (Finkenrath, Knechtli, Leder, "Application of Domain Decomposition to the
 * Evaluation of Fermion Determinant Ratios", Lattice 2012; Sec. 1, Eq. 1)
 *
 *     D = [[D_bb, D_bw], [D_wb, D_ww]],  det D = det Dhat * det D_ww * det D_bb,
 *     Dhat = 1 - D_bb^-1 D_bw D_ww^-1 D_wb,   on range(P): Dhat^-1 = 1 - P Dc_bw D_wb
 *
 * and the two-flavour reweighting factor W_gl of Eq. (8), estimated with
 * complex Gaussian noise as prod_i (1/N_hit) sum_j exp(-eta_ij^+ (Mh_i^+ Mh_i - 1) eta_ij),
 * Mh_i = Dhat(m_i)^-1 Dhat(m_{i-1}), m_i linear in m between m1 and m2 (Sec. 2, 2.1).
 *
 * Operator (mass normalisation; Eq. 6 needs D(m1) = D(m2) + (m1 - m2)):
 *     D(m) = (4 + m) + c_sw (i/4) sum sigma_{mu nu} Fhat_{mu nu} - 1/2 H,   m = 1/(2 kappa) - 4,
 * H the Wilson hopping term with (1 -+ gamma_mu) projectors, chiral gamma basis,
 * clover-leaf Fhat = (Q - Q^+)/8, hops across the time boundary times time_bc.
 *
 * Conventions at this boundary (all FP64 complex, interleaved re/im):
 *   site index  x = ((x0*L1 + x1)*L2 + x2)*L3 + x3, x0 = time (extent lat[0])
 *   spinor      [nrhs][V][4 spin][3 colour]   (16 bytes per complex entry)
 *   links       [4 mu][V][3][3], U_mu(x) = link from x to x + mu, row-major
 *   colour of a Schwarz block: (sum_mu x_mu / blk_mu) mod 2, black = 0;
 *   P = black sites with a nearest neighbour in another block (all 12 components).
 *   Schur-space vectors are full-lattice spinors that are zero off range(P).
 *
 * Ownership: every data pointer is a caller-owned DEVICE buffer (e.g. a torch
 * tensor's data_ptr) unless its name ends in _host.  The library copies the links
 * at create time, never frees caller memory, and owns its workspace (allocated on
 * first use, freed by ddwc_destroy).  `stream` is a hipStream_t (NULL = default).
 *
 * Errors: every function returns a ddwc_status.  Argument and geometry errors
 * (DDWC_EINVAL) are detected on the host before any launch and nothing is written.
 * ddwc_last_error() gives a thread-local message for the last non-zero status.
 * Calls that fill a ddwc_stats synchronise their stream; ddwc_dslash_apply is
 * asynchronous.  Calls on one context must not overlap (they share workspace).
 */
#ifndef DDWC_H
#define DDWC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ddwc_ctx ddwc_ctx;

typedef enum {
    DDWC_OK = 0,
    DDWC_EINVAL = -1,     /* bad argument or geometry; nothing launched */
    DDWC_ENOCONV = -2,    /* a solve hit maxit; best iterate written, stats filled */
    DDWC_EHIP = -3,       /* HIP runtime error */
    DDWC_ENONFINITE = -4, /* NaN or Inf met in a residual or norm */
    DDWC_EUNDEF = -5      /* estimate undefined: non-finite step mean or variance */
} ddwc_status;

/* DDWC_MIXED16: as DDWC_MIXED32, except that the inner BiCGStab of the even-odd global solver
 * and of the even-odd Schwarz block solver keeps its vectors in FP16 with one FP32 scale per
 * site and RHS, and its links in FP16 (clover, arithmetic and the solution correction in
 * FP32; FP64 defect correction restores the tolerance).  ddwc_dslash_apply, lattices with an
 * odd block extent, and block solves on blocks that the LDS-resident inner kernel takes
 * (DDWC_OPT_BLOCK_KERNEL) run as DDWC_MIXED32.  At most 256 RHS per call in the global solver. */
typedef enum { DDWC_FP64 = 0, DDWC_MIXED32 = 1, DDWC_MIXED16 = 2 } ddwc_precision;
typedef enum { DDWC_BLACK = 0, DDWC_WHITE = 1 } ddwc_colour;
typedef enum { DDWC_OP_FULL = 0, DDWC_OP_SCHUR = 1 } ddwc_operator;

typedef struct {
    int outer_iters;     /* FP64 defect-correction steps (restarts for DDWC_FP64) */
    int inner_iters;     /* Krylov iterations summed over restarts (max over RHS / blocks) */
    double rel_residual; /* final ||b - A x|| / ||b|| in FP64, max over RHS (and blocks) */
    double seconds;      /* host wall time of the call */
} ddwc_stats;

/*
 * Create a context for one gauge field.
 *   lat[4]    = {T, L1, L2, L3};  blk[4] = Schwarz block extents (Sec. 1).
 *   Geometry: blk[mu] divides lat[mu], and lat[mu]/blk[mu] is even and >= 2.
 *   time_bc   = -1 (antiperiodic) or +1 (periodic) in time; space is periodic.
 *   c_sw      = clover coefficient (0 gives plain Wilson).
 *   links_dev = canonical links (device, read during the call).
 * Builds the clover term on the device (once per configuration).
 */
int ddwc_create(ddwc_ctx **ctx, const int lat[4], const int blk[4], int time_bc, double c_sw,
                const void *links_dev, void *stream);
int ddwc_destroy(ddwc_ctx *ctx);

/*
 * out = D(m) in for nrhs right-hand sides (the Wilson-clover operator of Sec. 1/2,
 * m = 1/(2 kappa) - 4).  prec = DDWC_FP64 computes in FP64; DDWC_MIXED32 rounds the
 * fields to FP32 and computes in FP32 (result returned in FP64).  Asynchronous.
 */
int ddwc_dslash_apply(ddwc_ctx *ctx, double kappa, const void *in, void *out, int nrhs, int prec, void *stream);

/*
 * ddwc_dslash_apply for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same operator and result, bit for
 * bit, with the internal-layout fields in a static device array of the library (256 MiB per GPU,
 * held until the process ends) instead of the context's workspace.  The call allocates nothing
 * and creates no events.  EINVAL (nothing launched) when the two fields need more than 256 MiB:
 * 2 x nrhs x V x 192 bytes for DDWC_FP64, 2 x nrhs x V x 96 bytes otherwise (at 48x24^3: one FP64
 * RHS, two FP32 RHS).  Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents: calls that overlap in time on one GPU (other streams, other threads, other contexts)
 * race and must be serialised by the caller.  Asynchronous on `stream`.
 */
int ddwc_dslash_apply_noalloc(ddwc_ctx *ctx, double kappa, const void *in, void *out, int nrhs, int prec,
                              void *stream);

/*
 * sol = D_cc(m)^-1 rhs for all Schwarz blocks of one colour (D_bb or D_ww: the
 * Dirichlet block operators on the diagonal, Sec. 1).  Only sites of that colour
 * are read; the other colour of sol is set to zero.  One persistent launch: one
 * workgroup per (block, rhs) iterates to ||r_k|| <= tol ||b_k|| for its own block.
 * prec = DDWC_MIXED32 runs FP32 BiCGStab inside FP64 defect correction.
 */
int ddwc_block_solve(ddwc_ctx *ctx, int colour, double kappa, const void *rhs, void *sol, int nrhs, double tol,
                     int maxit, int prec, ddwc_stats *stats, void *stream);

/*
 * Schur complement on range(P) (Sec. 1).  inverse = 0: out = Dhat_P(m) in
 * = P in - P D_bb^-1 D_bw D_ww^-1 D_wb P in (two block sweeps).  inverse = 1:
 * out = Dhat_P(m)^-1 in = P in - P [D(m)^-1 (0_b, D_wb P in)]_b (one global solve).
 * in is projected with P first; out is zero off range(P).
 */
int ddwc_schur_apply(ddwc_ctx *ctx, double kappa, int inverse, const void *in, void *out, int nrhs, double tol,
                     int prec, ddwc_stats *stats, void *stream);

/*
 * x = D(m)^-1 b, BiCGStab on all nrhs at once (multi-RHS Dslash), until
 * ||b - D x|| <= tol ||b|| in FP64 for every RHS.  prec = DDWC_MIXED32: FP32 inner
 * solves with FP64 defect correction (the FP64 residual is recomputed after each).
 */
int ddwc_solve(ddwc_ctx *ctx, double kappa, const void *b, void *x, int nrhs, double tol, int maxit, int prec,
               ddwc_stats *stats, void *stream);

/*
 * Determinant-ratio estimate (Eq. 3 for op = FULL, Eq. 8 for SCHUR; n_f = 1: Eq. 11).
 *   eta         = noise, device, [n_interp][n_hit][V][4][3] (complex Gaussian, E|eta_k|^2 = 1;
 *                 for SCHUR it is projected with P first).
 *   n_f = 2:  x_host = [n_interp][n_hit] exponents x_ij = eta^+ (M^+ M - 1) eta, computed in the
 *                 cancellation-free form x = 2 Re<eta, y> + ||y||^2 with y = M eta - eta;
 *             the estimate is of 1/det(M^+ M) = W for two degenerate flavours.
 *   n_f = 1:  x_host = [n_interp][n_hit][2] complex exponents (re, im) x_ij = eta^+ (M - 1) eta
 *                 = <eta, y>; the estimate is of 1/det M, and only the real part of each step's
 *                 sample mean is kept (the expectation is real by gamma_5-hermiticity).
 *   log_w_gl    = sum_i ln Re[(1/n_hit) sum_j exp(-x_ij)]   (FP64, log domain).
 *   step_var_host = [n_interp] relative sample variance var_j(w)/mean_j(w)^2 of the weights
 *                 w_j = Re exp(-x_ij).  May be null.
 * Masses m_i = (i/N) m2 + ((N-i)/N) m1 linear in m (Sec. 2.1); all n_hit noise vectors of
 * a step go through the solvers as one multi-RHS batch; both flavour numbers use the same
 * solves.  Returns DDWC_EUNDEF (x_host filled, *log_w_gl = NaN) when a step's real mean is
 * not positive or a mean or variance is not finite.
 */
int ddwc_det_ratio_estimate(ddwc_ctx *ctx, double kappa1, double kappa2, int n_interp, int op, int n_f,
                            const void *eta, int n_hit, double tol, int prec, double *x_host, double *log_w_gl,
                            double *step_var_host, ddwc_stats *stats, void *stream);

/*
 * Nested domain decomposition (Sec. 2.2: the 8^4 blocks of the larger lattice are split again
 * into an 8^4 Schur complement with Dirichlet boundaries and 4^4 blocks).
 *   outer: the context whose Schwarz blocks B are split; inner: a context of the same lattice,
 *   links, c_sw and time boundary with blocks b, b_mu dividing B_mu (EINVAL otherwise; the links
 *   are compared through a fingerprint taken at ddwc_create).
 * For the outer blocks of one colour, A = D_cc (the direct sum of their Dirichlet operators,
 * Sec. 1) splits by the inner blocks (inner colouring) as det A = det Ahat * prod_s det D_s,
 *   Ahat = 1 - A_bb^-1 A_bw A_ww^-1 A_wb on range(P_c),
 * P_c = the face sites of black inner blocks inside the colour's outer blocks.  This call
 * estimates log |det Ahat(m2) / det Ahat(m1)|^2 (n_f = 2; n_f = 1: the one-flavour form) exactly
 * as ddwc_det_ratio_estimate(op = SCHUR) estimates W_gl (Eq. 8, mass interpolation, log domain):
 * x_ij from e = P_c eta_ij, with Ahat^-1 applied by one block solve of the outer context.
 * Arguments after colour as in ddwc_det_ratio_estimate (eta canonical, n_hit RHS per step,
 * x_host [n_interp][n_hit], pairs for n_f = 1).  stats: the outer block solves.  The full
 * log W of the larger lattice is log W_gl (outer context) + the two colours of this call
 * + 2 sum over all inner blocks of [ln|det D_s(m2)| - ln|det D_s(m1)|] (ddwc_block_logdet
 * on the inner context).  Uses both contexts' workspace; synchronises the stream.
 */
int ddwc_det_ratio_nested(ddwc_ctx *outer, ddwc_ctx *inner, int colour, double kappa1, double kappa2,
                          int n_interp, int n_f, const void *eta, int n_hit, double tol, int prec, double *x_host,
                          double *log_w, double *step_var_host, ddwc_stats *stats, void *stream);

/*
 * Derivatives of the two-flavour exponents (Eq. 3 / Eq. 8 as in ddwc_det_ratio_estimate).
 * Given the upstream gradient gx_host = dL/dx_ij [n_interp][n_hit] of any scalar L of the
 * exponents (e.g. L = log W_gl: gx_ij = -softmax_j(-x_ij)), returns
 *   *dkappa2_host = dL/dkappa2 (through m2 = 1/(2 kappa2) - 4 and the interpolation masses
 *                   m_i, linear in m), if dkappa2_host is not null;
 *   dU            = dL/dRe U + i dL/dIm U for every link matrix (device, canonical
 *                   [4][V][3][3] complex128, overwritten; hop and clover terms), if not null.
 * The solves of the forward pass are recomputed (nothing is stored between calls); the
 * adjoint solves use D^+ = g5 D g5 and Dhat^+ = g5 Dhat g5.  Same eta, n_hit, tol, prec
 * and geometry rules as ddwc_det_ratio_estimate; two flavours only.
 */
int ddwc_det_ratio_grad(ddwc_ctx *ctx, double kappa1, double kappa2, int n_interp, int op, const void *eta,
                        int n_hit, double tol, int prec, const double *gx_host, double *dkappa2_host, void *dU,
                        ddwc_stats *stats, void *stream);

/*
 * Link derivative of F = sum_r w_host[r] Re <a_r, D b_r> (the force term an adjoint pass
 * or an HMC step needs): dU = dF/dRe U + i dF/dIm U, hop and clover terms, device canonical
 * [4][V][3][3] complex128, overwritten.  a, b: device, canonical [nrhs][V][4][3] complex128.
 * Independent of the mass.  Synchronises the stream.
 */
int ddwc_link_force(ddwc_ctx *ctx, const void *a, const void *b, int nrhs, const double *w_host, void *dU,
                    void *stream);

/*
 * Exact ln|det D_k(m)| and sign of every Dirichlet Schwarz block k of one colour (the block
 * factor of Eq. 7: det D = det Dhat * det D_bb * det D_ww, D_bb and D_ww the direct sums of
 * the D_k).  logabs_host [NBc], sign_host [NBc] (may be null), in the library's block order:
 * blocks of the colour sorted by block coordinates (n_0, n_1, n_2, n_3) lexicographically.
 * With every block extent even the odd sites are eliminated first (det D_k = prod det A_oo *
 * det M_k), so the dense LU has dimension 6 Vb; otherwise 12 Vb.  EINVAL if one dense block
 * exceeds 16 GiB; EUNDEF if a block is singular or its determinant is not real to 1e-6.
 * Synchronises the stream.
 */
int ddwc_block_logdet(ddwc_ctx *ctx, double kappa, int colour, double *logabs_host, int *sign_host, void *stream);

/*
 * The block factor of the two-flavour log W (Eq. 7: det D = det Dhat * det D_bb * det D_ww):
 *   *out_host = 2 sum_k [ln|det D_k(m2)| - ln|det D_k(m1)|] over the blocks of both colours,
 * from four ddwc_block_logdet calls (same limits and errors).  Synchronises the stream.
 */
int ddwc_log_w_blocks(ddwc_ctx *ctx, double kappa1, double kappa2, double *out_host, void *stream);

/*
 * Combination of given exponents, on the host (no context, no device work): Eq. (8) per step
 * for n_f = 2, Eq. (11) with the real part of each step's mean for n_f = 1, exactly as
 * ddwc_det_ratio_estimate combines its own exponents.
 *   x_host        [n_interp][n_hit] (n_f = 2) or [n_interp][n_hit][2] (n_f = 1, re/im pairs)
 *   log_w         sum_i ln Re[(1/n_hit) sum_j exp(-x_ij)] (NaN with DDWC_EUNDEF)
 *   step_var_host [n_interp] relative sample variances (N_hit - 1 in the denominator); may be null
 *   gx_host       [n_interp][n_hit] d log_w / d x_ij = -exp(-x_ij) / sum_j exp(-x_ij) (n_f = 2
 *                 only, EINVAL otherwise); may be null.  This is the upstream gradient that
 *                 ddwc_det_ratio_grad takes for L = log W_gl.
 * EINVAL for non-finite exponents or bad sizes; EUNDEF when a step's real mean is not positive
 * or a mean or variance is not finite.
 */
int ddwc_log_w_combine(const double *x_host, int n_interp, int n_hit, int n_f, double *log_w, double *step_var_host,
                       double *gx_host);

/*
 * Total two-flavour log W with nested domain decomposition (Sec. 2.2):
 *   parts_host[0] = log W_gl of the outer context (ddwc_det_ratio_estimate, op = SCHUR, eta_gl,
 *                   n_hit_gl noise vectors per step);
 *   parts_host[1], [2] = the nested factors of the black and white outer blocks
 *                   (ddwc_det_ratio_nested with eta_black, eta_white, n_hit_nested per step);
 *   parts_host[3] = the exact block factor of the inner blocks (ddwc_log_w_blocks on inner);
 *   parts_host[4] = their sum, log W.
 * Every eta is canonical [n_interp][n_hit][V][4][3] on the device.  Same rules and errors as the
 * calls it makes; stats: the global solves of parts_host[0].  Synchronises the stream.
 */
int ddwc_log_w_nested_total(ddwc_ctx *outer, ddwc_ctx *inner, double kappa1, double kappa2, int n_interp,
                            const void *eta_gl, int n_hit_gl, const void *eta_black, const void *eta_white,
                            int n_hit_nested, double tol, int prec, double *parts_host, ddwc_stats *stats,
                            void *stream);

/*
 * Schedule options of a context.
 *   DDWC_OPT_GRAPHS        1: the global solver replays each chunk of BiCGStab iterations from
 *                          a captured HIP graph (cached per buffer set and mass; not while
 *                          profiling); 0: launches them one by one.  Default 1.
 *   DDWC_OPT_POLL          iterations between the host's convergence checks, [1, 64]; default 2.
 *   DDWC_OPT_BLOCK_THREADS workgroup size of the Schwarz block kernels: 0 (enough waves for one
 *                          block parity, at most 768 for the FP32/FP16 inner solver and 256 for
 *                          the FP64 kernels) or a multiple of 64 in [64, 768] (capped alike).
 *   DDWC_OPT_SOLVER        global solver: 0 even-odd BiCGStab (default; lexicographic BiCGStab when
 *                          a block extent is odd), 1 GCR (8 directions per cycle, restarted with
 *                          the exact FP64 residual) preconditioned by the Schwarz alternating
 *                          procedure: 3 multiplicative cycles over the black then the white
 *                          blocks, each block solve by the persistent block solver to 1e-1.
 *   DDWC_OPT_BLOCK_LDS     KiB of LDS reserved (not used) by each global-memory block-solver workgroup,
 *                          which caps the workgroups resident per CU and so the block vectors in
 *                          flight (0 = none; at most the device's per-workgroup LDS minus 1 KiB).
 *   DDWC_OPT_BLOCK_KERNEL  inner solver of the even-odd Schwarz block solves in DDWC_MIXED32 and
 *                          DDWC_MIXED16: 0 (default) the LDS-resident FP32 kernel wherever a block
 *                          parity has at most 768 sites and its two staged fields fit the LDS (both
 *                          precisions then run it, FP32 storage); 1 the global-memory kernel.
 *   DDWC_OPT_INNER_FLOOR   the FP32 inner BiCGStab of the even-odd global solver (DDWC_MIXED32) stops
 *                          at a relative residual of at least value x 1e-8 before the FP64 defect
 *                          correction restarts it, in [1, 100000]; default 200 (2e-6).
 *   DDWC_OPT_OP_THREADS    workgroup size of the RHS-innermost operator kernels (the even-odd
 *                          global solver's, and ddwc_dslash_apply's with several FP32 RHS): 128,
 *                          256 (default) or 512; a value below the RHS count runs 256.
 *   DDWC_OPT_TILE_ORDER    dispatch order of those kernels' workgroups: 0 site index order;
 *                          1 (default) interleaved by Schwarz-block rank, so that face-adjacent blocks
 *                          of the two colours run on the same XCD at about the same time (not in
 *                          ddwc_dslash_apply_noalloc, which builds no order table).  Neither option
 *                          changes a result of ddwc_dslash_apply.
 * Results do not depend on the graph and LDS options; the others can change iteration counts and
 * rounding, never the tolerance reached.  EINVAL for unknown options or values.
 */
typedef enum {
    DDWC_OPT_GRAPHS = 0,
    DDWC_OPT_POLL = 1,
    DDWC_OPT_BLOCK_THREADS = 2,
    DDWC_OPT_SOLVER = 3,
    DDWC_OPT_BLOCK_LDS = 4,
    DDWC_OPT_BLOCK_KERNEL = 5,
    DDWC_OPT_INNER_FLOOR = 6,
    DDWC_OPT_OP_THREADS = 7,
    DDWC_OPT_TILE_ORDER = 8
} ddwc_option;
int ddwc_set_option(ddwc_ctx *ctx, int option, int value);
int ddwc_get_option(ddwc_ctx *ctx, int option, int *value);

/*
 * Autotuner: times the schedule options on this lattice with nrhs reproducible right-hand
 * sides at the given kappa and precision, tolerance 1e-8, and sets the fastest of each group in
 * turn: the block inner solver on a block sweep of one colour (DDWC_OPT_BLOCK_KERNEL 0 where it
 * applies; kernel 1 at each DDWC_OPT_BLOCK_THREADS in {0, 128, 256, 512} without and with the
 * LDS reservations that leave room for 2 or 4 block-solver workgroups per CU); then, on a global
 * solve, DDWC_OPT_OP_THREADS in {128, 256, 512} with each DDWC_OPT_TILE_ORDER; then each poll
 * interval in {2, 4, 8} with and without graphs.  *seconds_host (may be null) receives the
 * tuning time.  Synchronises.
 */
int ddwc_autotune(ddwc_ctx *ctx, double kappa, int nrhs, int prec, double *seconds_host, void *stream);

/*
 * Kernel timing for measurement.  When enabled, launches of the library's kernels
 * are bracketed with HIP events on their stream; ddwc_profile_read synchronises and
 * returns, for kernel class `kclass` (DDWC_K_*), the number of launches and their
 * summed duration in milliseconds since the last reset, and in *bytes the algorithmic HBM
 * bytes of the operator classes' launches.  For DDWC_K_BLOCK, whose kernels work from LDS and
 * the caches, *bytes holds instead the model's floating-point operation count (per inner
 * iteration and even site: two block-operator applications over both parities at 180 flops per
 * in-block hop and 540 per site for the clover, plus 400 for the vector updates).
 */
typedef enum {
    DDWC_K_DSLASH64 = 0,  /* full-lattice Dslash, FP64 */
    DDWC_K_DSLASH32 = 1,  /* Dslash in FP32/FP16: full lattice, and the diagonal-and-hop half of the
                             even-odd operator in the global solver */
    DDWC_K_BLOCK = 2,     /* persistent block solver */
    DDWC_K_BLAS = 3,      /* vector updates and reductions */
    DDWC_K_OTHER = 4,     /* hops, conversions, projections */
    DDWC_K_EOHOP = 5,     /* hop-and-inverse half of the even-odd operator in the FP32/FP16 global solver */
    DDWC_K_COUNT = 6
} ddwc_kernel_class;
int ddwc_profile_enable(ddwc_ctx *ctx, int on);
int ddwc_profile_read(ddwc_ctx *ctx, int kclass, long long *launches, double *total_ms, double *bytes);

/*
 * Streaming reference: dst = src for `bytes` bytes (device buffers, 16-byte aligned, bytes a multiple
 * of 16; they must not overlap), by the library's own copy kernel (float4 words, four loads in flight
 * per thread, grid-stride rounds).  Its rate is the practical HBM streaming ceiling that the operator
 * kernels are measured against beside the nominal peak; with a known size it also calibrates memory
 * counters.  Asynchronous on `stream`; needs no context.
 */
int ddwc_stream_copy(const void *src, void *dst, size_t bytes, void *stream);

/* Algorithmic HBM bytes of one full-lattice Dslash launch at this geometry (per RHS count). */
double ddwc_dslash_bytes(const ddwc_ctx *ctx, int nrhs, int prec);

const char *ddwc_last_error(void);
const char *ddwc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DDWC_H */

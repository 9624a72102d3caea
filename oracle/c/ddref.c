/*
 * Matrix-free FP64 reference of the Wilson-clover operator, Schwarz block
 * solves and the two-flavour estimator exponent, in plain C99 + OpenMP.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test-suite for lattices too large for
 * the assembled-matrix oracle, and timed as the CPU baseline.  It shares no
 * code with the HIP library.
 *
 * Operator (mass normalisation; the paper relies on D(m1) = D(m2) + dm, Eq. 6):
 *   (D psi)(x) = (4+m) psi(x) + C(x) psi(x)
 *                - 1/2 sum_mu [(1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^+ psi(x-mu)]
 *   C(x) = c_sw (i/4) sum_{mu != nu} sigma_{mu nu} Fhat_{mu nu}(x), Fhat = (Q - Q^+)/8,
 * chiral gamma matrices, hops across the time boundary times time_bc.
 * Written with full 4x4 spin matrices and a full 12x12 clover per site.
 *
 * Schwarz (Sec. 1): block coordinate n = x / b, colour = sum(n) mod 2, black = 0;
 * D_cc keeps only hops inside a block; D_wb, D_bw are the hops between colours;
 * P = black sites with a neighbour in another block.
 *
 * Layouts: spinor [V][4][3], links [4][V][3][3], complex double, x3 fastest.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

typedef struct {
    int lat[4], blk[4], tbc;
    long V;
    double csw;
    cplx *U;     /* [4][V][3][3] */
    cplx *C;     /* [V][12][12] clover term (mass-free) */
    int *colour; /* per site */
    long *bid;   /* block number per site */
    char *pmask; /* per site: black face site */
    cplx g[4][4][4];
} ref_t;

static void coords_of(const ref_t *h, long s, int c[4]) {
    c[3] = (int)(s % h->lat[3]); s /= h->lat[3];
    c[2] = (int)(s % h->lat[2]); s /= h->lat[2];
    c[1] = (int)(s % h->lat[1]); s /= h->lat[1];
    c[0] = (int)s;
}

static long index_of(const ref_t *h, const int c[4]) {
    int d[4];
    for (int k = 0; k < 4; k++) d[k] = ((c[k] % h->lat[k]) + h->lat[k]) % h->lat[k];
    return (((long)d[0] * h->lat[1] + d[1]) * h->lat[2] + d[2]) * h->lat[3] + d[3];
}

/* neighbour x + step*mu and the boundary factor of that hop */
static long nbr(const ref_t *h, long s, int mu, int step, double *fac) {
    int c[4];
    coords_of(h, s, c);
    c[mu] += step;
    *fac = 1.0;
    if (mu == 0 && (c[0] < 0 || c[0] >= h->lat[0])) *fac = (double)h->tbc;
    return index_of(h, c);
}

static const cplx *link(const ref_t *h, int mu, long s) { return h->U + ((long)mu * h->V + s) * 9; }

static void mat_mul(const cplx *a, const cplx *b, cplx *o) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cplx t = 0;
            for (int k = 0; k < 3; k++) t += a[3 * i + k] * b[3 * k + j];
            o[3 * i + j] = t;
        }
}

static void mat_dag(const cplx *a, cplx *o) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) o[3 * i + j] = conj(a[3 * j + i]);
}

static void mat_prod4(const cplx *a, const cplx *b, const cplx *c, const cplx *d, cplx *o) {
    cplx t1[9], t2[9];
    mat_mul(a, b, t1);
    mat_mul(t1, c, t2);
    mat_mul(t2, d, o);
}

static void build_gamma(ref_t *h) {
    memset(h->g, 0, sizeof(h->g));
    /* g0 = [[0,-1],[-1,0]] */
    h->g[0][0][2] = h->g[0][1][3] = h->g[0][2][0] = h->g[0][3][1] = -1;
    /* gk = [[0, -i s_k], [i s_k, 0]] */
    cplx s[3][2][2] = {{{0, 1}, {1, 0}}, {{0, -I}, {I, 0}}, {{1, 0}, {0, -1}}};
    for (int k = 0; k < 3; k++)
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                h->g[k + 1][a][b + 2] = -I * s[k][a][b];
                h->g[k + 1][a + 2][b] = I * s[k][a][b];
            }
}

/* Q_{mu nu}(x), the four plaquette leaves at x */
static void plaq_sum(const ref_t *h, long x, int mu, int nu, cplx *q) {
    double f;
    long xpm = nbr(h, x, mu, 1, &f), xpn = nbr(h, x, nu, 1, &f);
    long xmm = nbr(h, x, mu, -1, &f), xmn = nbr(h, x, nu, -1, &f);
    long xmm_pn = nbr(h, xmm, nu, 1, &f), xmm_mn = nbr(h, xmm, nu, -1, &f);
    long xpm_mn = nbr(h, xpm, nu, -1, &f);
    cplx d1[9], d2[9], l[9];
    for (int i = 0; i < 9; i++) q[i] = 0;
    mat_dag(link(h, mu, xpn), d1);
    mat_dag(link(h, nu, x), d2);
    mat_prod4(link(h, mu, x), link(h, nu, xpm), d1, d2, l);
    for (int i = 0; i < 9; i++) q[i] += l[i];
    mat_dag(link(h, mu, xmm_pn), d1);
    mat_dag(link(h, nu, xmm), d2);
    mat_prod4(link(h, nu, x), d1, d2, link(h, mu, xmm), l);
    for (int i = 0; i < 9; i++) q[i] += l[i];
    mat_dag(link(h, mu, xmm), d1);
    mat_dag(link(h, nu, xmm_mn), d2);
    mat_prod4(d1, d2, link(h, mu, xmm_mn), link(h, nu, xmn), l);
    for (int i = 0; i < 9; i++) q[i] += l[i];
    mat_dag(link(h, nu, xmn), d1);
    mat_dag(link(h, mu, x), d2);
    mat_prod4(d1, link(h, mu, xmn), link(h, nu, xpm_mn), d2, l);
    for (int i = 0; i < 9; i++) q[i] += l[i];
}

static void build_clover(ref_t *h) {
#pragma omp parallel for schedule(static)
    for (long x = 0; x < h->V; x++) {
        cplx *c = h->C + x * 144;
        for (int i = 0; i < 144; i++) c[i] = 0;
        if (h->csw == 0.0) continue;
        for (int mu = 0; mu < 4; mu++)
            for (int nu = 0; nu < 4; nu++) {
                if (mu == nu) continue;
                cplx q[9], F[9], sig[4][4];
                plaq_sum(h, x, mu, nu, q);
                for (int a = 0; a < 3; a++)
                    for (int b = 0; b < 3; b++) F[3 * a + b] = (q[3 * a + b] - conj(q[3 * b + a])) / 8.0;
                for (int s = 0; s < 4; s++)
                    for (int t = 0; t < 4; t++) {
                        cplx gg = 0;
                        for (int k = 0; k < 4; k++) gg += h->g[mu][s][k] * h->g[nu][k][t] - h->g[nu][s][k] * h->g[mu][k][t];
                        sig[s][t] = 0.5 * I * gg;
                    }
                for (int s = 0; s < 4; s++)
                    for (int a = 0; a < 3; a++)
                        for (int t = 0; t < 4; t++)
                            for (int b = 0; b < 3; b++)
                                c[(3 * s + a) * 12 + 3 * t + b] += h->csw * 0.25 * I * sig[s][t] * F[3 * a + b];
            }
    }
}

ref_t *ref_create(const int *lat, const int *blk, int tbc, double csw, const cplx *links) {
    ref_t *h = (ref_t *)calloc(1, sizeof(ref_t));
    memcpy(h->lat, lat, sizeof(h->lat));
    memcpy(h->blk, blk, sizeof(h->blk));
    h->tbc = tbc;
    h->csw = csw;
    h->V = (long)lat[0] * lat[1] * lat[2] * lat[3];
    h->U = (cplx *)malloc(sizeof(cplx) * 36 * h->V);
    memcpy(h->U, links, sizeof(cplx) * 36 * h->V);
    h->C = (cplx *)malloc(sizeof(cplx) * 144 * h->V);
    h->colour = (int *)malloc(sizeof(int) * h->V);
    h->bid = (long *)malloc(sizeof(long) * h->V);
    h->pmask = (char *)malloc(h->V);
    build_gamma(h);
    for (long x = 0; x < h->V; x++) {
        int c[4], n[4], sum = 0, face = 0;
        coords_of(h, x, c);
        long b = 0;
        for (int k = 0; k < 4; k++) {
            n[k] = c[k] / blk[k];
            sum += n[k];
            b = b * (lat[k] / blk[k]) + n[k];
            int r = c[k] % blk[k];
            if (r == 0 || r == blk[k] - 1) face = 1;
        }
        h->colour[x] = sum % 2;
        h->bid[x] = b;
        h->pmask[x] = (char)(face && h->colour[x] == 0);
    }
    build_clover(h);
    return h;
}

void ref_destroy(ref_t *h) {
    if (!h) return;
    free(h->U); free(h->C); free(h->colour); free(h->bid); free(h->pmask);
    free(h);
}

void ref_clover(const ref_t *h, cplx *out) { memcpy(out, h->C, sizeof(cplx) * 144 * h->V); }

/*
 * Generic masked application.  Output sites: all (out_colour < 0) or one colour.
 * hops: 0 = none, 1 = all, 2 = only inside the block, 3 = only to other blocks.
 * diag: include (4+m) + C.  Output sites not selected are set to 0.
 */
static void apply_masked(const ref_t *h, double m, int out_colour, int hops, int diag, const cplx *in, cplx *out) {
#pragma omp parallel for schedule(static)
    for (long x = 0; x < h->V; x++) {
        cplx acc[12];
        for (int i = 0; i < 12; i++) acc[i] = 0;
        if (out_colour < 0 || h->colour[x] == out_colour) {
            const cplx *px = in + 12 * x;
            if (diag) {
                const cplx *c = h->C + 144 * x;
                for (int i = 0; i < 12; i++) {
                    cplx t = (4.0 + m) * px[i];
                    for (int j = 0; j < 12; j++) t += c[12 * i + j] * px[j];
                    acc[i] = t;
                }
            }
            if (hops)
                for (int mu = 0; mu < 4; mu++)
                    for (int dir = 0; dir < 2; dir++) {
                        int step = dir == 0 ? 1 : -1;
                        double fac;
                        long y = nbr(h, x, mu, step, &fac);
                        int same = h->bid[y] == h->bid[x];
                        if ((hops == 2 && !same) || (hops == 3 && same)) continue;
                        cplx W[9];
                        if (step == 1)
                            memcpy(W, link(h, mu, x), sizeof(W));
                        else
                            mat_dag(link(h, mu, y), W);
                        const cplx *py = in + 12 * y;
                        cplx up[12]; /* U psi(y) per spin */
                        for (int s = 0; s < 4; s++)
                            for (int a = 0; a < 3; a++) {
                                cplx t = 0;
                                for (int b = 0; b < 3; b++) t += W[3 * a + b] * py[3 * s + b];
                                up[3 * s + a] = t;
                            }
                        double sg = step == 1 ? -1.0 : 1.0; /* (1 - g) forward, (1 + g) backward */
                        for (int s = 0; s < 4; s++)
                            for (int a = 0; a < 3; a++) {
                                cplx t = up[3 * s + a];
                                for (int k = 0; k < 4; k++) t += sg * h->g[mu][s][k] * up[3 * k + a];
                                acc[3 * s + a] += -0.5 * fac * t;
                            }
                    }
        }
        for (int i = 0; i < 12; i++) out[12 * x + i] = acc[i];
    }
}

void ref_dslash(const ref_t *h, double m, const cplx *in, cplx *out) { apply_masked(h, m, -1, 1, 1, in, out); }

/* D_cc psi: the Dirichlet block operators of one colour */
void ref_block_apply(const ref_t *h, int colour, double m, const cplx *in, cplx *out) {
    apply_masked(h, m, colour, 2, 1, in, out);
}

/* hops into colour to_colour from the other colour: D_wb (to_colour = 1) or D_bw (0) */
void ref_hop(const ref_t *h, int to_colour, const cplx *in, cplx *out) {
    apply_masked(h, 0.0, to_colour, 3, 0, in, out);
}

/* ----------------------------------------------------------------- vector helpers */
static cplx dot(long n, const cplx *a, const cplx *b) {
    double re = 0, im = 0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
    for (long i = 0; i < n; i++) {
        cplx t = conj(a[i]) * b[i];
        re += creal(t);
        im += cimag(t);
    }
    return re + I * im;
}

static double nrm2(long n, const cplx *a) { return creal(dot(n, a, a)); }

typedef void (*op_fn)(const ref_t *, int, double, const cplx *, cplx *);

/*
 * Optional bookkeeping of the solves done by ref_exponent, in call order: iterations and
 * wall seconds of each, and an iteration cap applied to each solve (0 = none).  Used to
 * time a bounded sample of one estimate.
 */
static int g_rec_on = 0, g_rec_n = 0, g_rec_cap = 0;
static int g_rec_iters[16];
static double g_rec_secs[16];

#include <omp.h>

static void op_full(const ref_t *h, int c, double m, const cplx *in, cplx *out) {
    (void)c;
    ref_dslash(h, m, in, out);
}

/*
 * BiCGStab (van der Vorst 1992) restarted from the true residual until
 * ||b - A x|| <= tol ||b||.  Returns total iterations, or -1 if not reached.
 */
static int bicgstab(const ref_t *h, op_fn A, int c, double m, const cplx *b, cplx *x, double tol, int maxit) {
    long n = 12 * h->V;
    cplx *r = malloc(sizeof(cplx) * n), *rh = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n);
    cplx *v = malloc(sizeof(cplx) * n), *s = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n);
    double bn = sqrt(nrm2(n, b));
    int it = 0, ok = 0;
    for (long i = 0; i < n; i++) x[i] = 0;
    if (bn == 0) { ok = 1; goto done; }
    for (int restart = 0; restart < 50 && it < maxit; restart++) {
        A(h, c, m, x, t);
        for (long i = 0; i < n; i++) { r[i] = b[i] - t[i]; rh[i] = r[i]; p[i] = r[i]; }
        double rn = sqrt(nrm2(n, r));
        if (rn <= tol * bn) { ok = 1; break; }
        cplx rho = dot(n, rh, r);
        for (; it < maxit; it++) {
            A(h, c, m, p, v);
            cplx alpha = rho / dot(n, rh, v);
            for (long i = 0; i < n; i++) s[i] = r[i] - alpha * v[i];
            A(h, c, m, s, t);
            cplx omega = dot(n, t, s) / nrm2(n, t);
            for (long i = 0; i < n; i++) {
                x[i] += alpha * p[i] + omega * s[i];
                r[i] = s[i] - omega * t[i];
            }
            rn = sqrt(nrm2(n, r));
            if (rn <= 0.1 * tol * bn) { it++; break; }
            cplx rho1 = dot(n, rh, r);
            cplx beta = (rho1 / rho) * (alpha / omega);
            rho = rho1;
            for (long i = 0; i < n; i++) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        }
    }
done:
    free(r); free(rh); free(p); free(v); free(s); free(t);
    return ok ? it : -1;
}

static int recorded(const ref_t *h, op_fn A, int c, double m, const cplx *b, cplx *x, double tol, int maxit) {
    if (!g_rec_on) return bicgstab(h, A, c, m, b, x, tol, maxit);
    double t0 = omp_get_wtime();
    int cap = g_rec_cap > 0 && g_rec_cap < maxit ? g_rec_cap : maxit;
    int it = bicgstab(h, A, c, m, b, x, tol, cap);
    if (g_rec_n < 16) {
        g_rec_secs[g_rec_n] = omp_get_wtime() - t0;
        g_rec_iters[g_rec_n] = it < 0 ? cap : it;
        g_rec_n++;
    }
    return g_rec_cap > 0 && it < 0 ? cap : it;
}

int ref_solve(const ref_t *h, double m, const cplx *b, cplx *x, double tol, int maxit) {
    return recorded(h, op_full, 0, m, b, x, tol, maxit);
}

int ref_block_solve(const ref_t *h, int colour, double m, const cplx *b, cplx *x, double tol, int maxit) {
    long n = 12 * h->V;
    cplx *bb = malloc(sizeof(cplx) * n);
    for (long s = 0; s < h->V; s++)
        for (int i = 0; i < 12; i++) bb[12 * s + i] = h->colour[s] == colour ? b[12 * s + i] : 0;
    int it = recorded(h, ref_block_apply, colour, m, bb, x, tol, maxit);
    free(bb);
    return it;
}

/* Start (cap >= 0) or read the solve record; returns the number of solves recorded. */
int ref_record(int on, int cap, int *iters, double *secs) {
    if (on) {
        g_rec_on = 1;
        g_rec_cap = cap;
        g_rec_n = 0;
        return 0;
    }
    g_rec_on = 0;
    for (int k = 0; k < g_rec_n; k++) {
        if (iters) iters[k] = g_rec_iters[k];
        if (secs) secs[k] = g_rec_secs[k];
    }
    return g_rec_n;
}

int ref_threads(void) { return omp_get_max_threads(); }

/* Thread count of the following parallel regions (timing only; results do not depend on it). */
void ref_set_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
}

static void mask_P(const ref_t *h, const cplx *in, cplx *out) {
    for (long s = 0; s < h->V; s++)
        for (int i = 0; i < 12; i++) out[12 * s + i] = h->pmask[s] ? in[12 * s + i] : 0;
}

/* Dhat_P phi = P phi - P D_bb^-1 D_bw D_ww^-1 D_wb P phi */
int ref_schur_apply(const ref_t *h, double m, const cplx *phi, cplx *out, double tol) {
    long n = 12 * h->V;
    cplx *e = malloc(sizeof(cplx) * n), *a = malloc(sizeof(cplx) * n), *b = malloc(sizeof(cplx) * n);
    mask_P(h, phi, e);
    ref_hop(h, 1, e, a);
    int i1 = ref_block_solve(h, 1, m, a, b, tol, 100000);
    ref_hop(h, 0, b, a);
    int i2 = ref_block_solve(h, 0, m, a, b, tol, 100000);
    for (long i = 0; i < n; i++) a[i] = e[i] - b[i];
    mask_P(h, a, out);
    free(e); free(a); free(b);
    return (i1 < 0 || i2 < 0) ? -1 : 0;
}

/* Dhat_P^-1 phi = P phi - P [D^-1 (0_b, D_wb P phi)]_b  (Sec. 1) */
int ref_schur_inverse(const ref_t *h, double m, const cplx *phi, cplx *out, double tol) {
    long n = 12 * h->V;
    cplx *e = malloc(sizeof(cplx) * n), *a = malloc(sizeof(cplx) * n), *chi = malloc(sizeof(cplx) * n);
    mask_P(h, phi, e);
    ref_hop(h, 1, e, a);
    int it = ref_solve(h, m, a, chi, tol, 100000);
    mask_P(h, chi, a);
    for (long i = 0; i < n; i++) out[i] = e[i] - a[i];
    free(e); free(a); free(chi);
    return it < 0 ? -1 : 0;
}

/*
 * Estimator exponent x = eta^+ (M^+ M - 1) eta of one noise vector (Eq. 3, Eq. 8).
 * op: 0 full M = D(m2)^-1 D(m1); 1 Schur Mh = Dhat_P(m2)^-1 Dhat_P(m1).
 * form: 0 plain ||M eta||^2 - ||eta||^2; 1 difference form (M eta - eta computed directly).
 */
int ref_exponent(const ref_t *h, int op, int form, double m1, double m2, const cplx *eta, double tol, double *x) {
    long n = 12 * h->V;
    double dm = m1 - m2;
    cplx *e = malloc(sizeof(cplx) * n), *a = malloc(sizeof(cplx) * n), *b = malloc(sizeof(cplx) * n);
    cplx *c = malloc(sizeof(cplx) * n), *d = malloc(sizeof(cplx) * n);
    int st = 0;
    if (op == 0) {
        memcpy(e, eta, sizeof(cplx) * n);
        if (form == 0) {
            ref_dslash(h, m1, e, a);
            st |= ref_solve(h, m2, a, b, tol, 100000) < 0;
            *x = nrm2(n, b) - nrm2(n, e);
        } else {
            st |= ref_solve(h, m2, e, b, tol, 100000) < 0;
            *x = 2 * dm * creal(dot(n, e, b)) + dm * dm * nrm2(n, b);
        }
    } else {
        mask_P(h, eta, e);
        if (form == 0) {
            st |= ref_schur_apply(h, m1, e, a, tol) != 0;
            st |= ref_schur_inverse(h, m2, a, b, tol) != 0;
            *x = nrm2(n, b) - nrm2(n, e);
        } else {
            /* g = dm P [D_bb1^-1 D_bb2^-1 D_bw D_ww1^-1 + D_bb2^-1 D_bw D_ww1^-1 D_ww2^-1] D_wb eta */
            ref_hop(h, 1, e, a);
            st |= ref_block_solve(h, 1, m1, a, b, tol, 100000) < 0;  /* b = w1 */
            st |= ref_block_solve(h, 1, m2, b, c, tol, 100000) < 0;  /* c = w12 */
            ref_hop(h, 0, b, a);
            st |= ref_block_solve(h, 0, m1, a, d, tol, 100000) < 0;  /* d = a1 */
            ref_hop(h, 0, c, a);
            for (long i = 0; i < n; i++) a[i] += d[i];
            st |= ref_block_solve(h, 0, m2, a, b, tol, 100000) < 0;
            for (long i = 0; i < n; i++) b[i] *= dm;
            mask_P(h, b, c);                                        /* c = g */
            st |= ref_schur_inverse(h, m2, c, d, tol) != 0;         /* d = zeta */
            *x = 2 * creal(dot(n, e, d)) + nrm2(n, d);
        }
    }
    free(e); free(a); free(b); free(c); free(d);
    return st ? -1 : 0;
}

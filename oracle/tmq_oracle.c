/*
 * tmq_oracle.c -- plain FP64 CPU reference of the Wilson twisted-mass operator,
 * its even/odd Schur complement and textbook conjugate gradient.
 *
 * TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the CPU
 * baseline of the benchmark use this file to judge the GPU library; the
 * library never calls it and the two share no code.  It is deliberately slow
 * and literal: dense 4x4 gamma matrices, dense 3x3 colour products, one
 * output site per loop iteration, no spin projection, no blocking.
 *
 * What is computed (J. & U., "tmLQCD", Appendix B eq. (eo0) -- the action in
 * the hopping-parameter form, r = 1 -- with the boundary phase of Sec. 4.1.2):
 *
 *   (H psi)(x) = sum_mu [ e^{+i theta_mu pi / L_mu} U(x,mu)      (1 + gamma_mu) psi(x+mu)
 *                       + e^{-i theta_mu pi / L_mu} U(x-mu,mu)^+ (1 - gamma_mu) psi(x-mu) ]
 *   M^{+-} = (1 +- i mut gamma_5) - kappa H           (tau^3 -> +-1, mut = 2 kappa mu)
 *   Q^{+-} = gamma_5 M^{+-}                            (eq. (eo1))
 *   Qhat^{+-} = gamma_5 ( M_oo^{+-} - M_oe (M_ee^{+-})^{-1} M_eo )   on odd sites (eq. (eo4))
 *   with M_eo = -kappa H restricted to even rows / odd columns (and M_oe the
 *   converse), and (M_ee^{+-})^{-1} = (1 -+ i mut gamma_5)/(1 + mut^2) (eq. (eo3)).
 *
 * The gamma matrices are those of Appendix A; gamma_5 = diag(1,1,-1,-1).
 * Directions: mu = 0:t, 1:x, 2:y, 3:z; gamma_mu is gamma_0..gamma_3.
 * Fields use the canonical host layout (site index ((t*LZ+z)*LY+y)*LX+x, then
 * spin, then colour; links (site, mu, row, column)); odd-site fields list the
 * odd sites ((t+x+y+z) odd) in increasing site index.
 *
 * CG (Sec. 4.4): textbook CG on a Hermitian positive definite operator A,
 * x_0 = 0, stopping when ||r||^2 < eps^2 (absolute) or ||r||^2/||b||^2 < eps^2
 * (relative) on the iterated residual.
 */
#define _GNU_SOURCE
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ---------------------------------------------------------------- gammas */

static cplx GAMMA[4][4][4]; /* gamma_0 .. gamma_3 */
static cplx GAMMA5[4][4];
static int gammas_ready = 0;

/* Appendix A, entries as (real, imaginary) pairs */
static const int G_RE[4][4][4] = {
    {{0, 0, -1, 0}, {0, 0, 0, -1}, {-1, 0, 0, 0}, {0, -1, 0, 0}},
    {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}},
    {{0, 0, 0, -1}, {0, 0, 1, 0}, {0, 1, 0, 0}, {-1, 0, 0, 0}},
    {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}},
};
static const int G_IM[4][4][4] = {
    {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}},
    {{0, 0, 0, -1}, {0, 0, -1, 0}, {0, 1, 0, 0}, {1, 0, 0, 0}},
    {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}},
    {{0, 0, -1, 0}, {0, 0, 0, 1}, {1, 0, 0, 0}, {0, -1, 0, 0}},
};

static void init_gammas(void)
{
    if (gammas_ready) return;
    for (int m = 0; m < 4; m++)
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++)
                GAMMA[m][i][j] = G_RE[m][i][j] + I * G_IM[m][i][j];
    memset(GAMMA5, 0, sizeof(GAMMA5));
    GAMMA5[0][0] = 1;
    GAMMA5[1][1] = 1;
    GAMMA5[2][2] = -1;
    GAMMA5[3][3] = -1;
    gammas_ready = 1;
}

/* export the matrices so the tests can check the Clifford algebra */
void orc_gammas(double *out /* 5 x 4 x 4 complex: gamma_0..3, gamma_5 */)
{
    init_gammas();
    cplx *o = (cplx *)out;
    for (int m = 0; m < 4; m++)
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++) o[(m * 4 + i) * 4 + j] = GAMMA[m][i][j];
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) o[(4 * 4 + i) * 4 + j] = GAMMA5[i][j];
}

/* ------------------------------------------------------------- geometry */

typedef struct {
    int ext[4]; /* T, LZ, LY, LX (memory order) */
    int L[4];   /* extent along mu = t, x, y, z */
    long V;
} geom;

static geom make_geom(const int *dims)
{
    geom g;
    for (int i = 0; i < 4; i++) g.ext[i] = dims[i];
    g.L[0] = dims[0]; /* t */
    g.L[1] = dims[3]; /* x */
    g.L[2] = dims[2]; /* y */
    g.L[3] = dims[1]; /* z */
    g.V = (long)dims[0] * dims[1] * dims[2] * dims[3];
    return g;
}

/* coordinates c[mu] (mu = t, x, y, z) of site index s */
static void coords(const geom *g, long s, int c[4])
{
    c[1] = (int)(s % g->L[1]);
    s /= g->L[1];
    c[2] = (int)(s % g->L[2]);
    s /= g->L[2];
    c[3] = (int)(s % g->L[3]);
    s /= g->L[3];
    c[0] = (int)s;
}

static long site_of(const geom *g, const int c[4])
{
    return (((long)c[0] * g->L[3] + c[3]) * g->L[2] + c[2]) * g->L[1] + c[1];
}

/* neighbour x + dir * mu-hat, periodic wrap (boundary phases enter the hop) */
static long neighbour(const geom *g, long s, int mu, int dir)
{
    int c[4];
    coords(g, s, c);
    c[mu] = (c[mu] + dir + g->L[mu]) % g->L[mu];
    return site_of(g, c);
}

static int parity(const geom *g, long s)
{
    int c[4];
    coords(g, s, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

/* list of odd sites in increasing site index; returns their number */
long orc_odd_sites(const int *dims, long *out)
{
    geom g = make_geom(dims);
    long k = 0;
    for (long s = 0; s < g.V; s++)
        if (parity(&g, s)) out[k++] = s;
    return k;
}

/* ------------------------------------------------------ small algebra */

/* out = (1 + sgn * gamma_mu) in, on spin, for every colour */
static void one_pm_gamma(int mu, int sgn, const cplx *in, cplx out[4][3])
{
    for (int i = 0; i < 4; i++)
        for (int c = 0; c < 3; c++) {
            cplx s = in[i * 3 + c];
            for (int j = 0; j < 4; j++) s += sgn * GAMMA[mu][i][j] * in[j * 3 + c];
            out[i][c] = s;
        }
}

/* out[spin] = U in[spin] (dag = 0) or U^+ in[spin] (dag = 1) */
static void colour_mul(const cplx *U, int dag, cplx in[4][3], cplx out[4][3])
{
    for (int i = 0; i < 4; i++)
        for (int a = 0; a < 3; a++) {
            cplx s = 0;
            for (int b = 0; b < 3; b++)
                s += (dag ? conj(U[b * 3 + a]) : U[a * 3 + b]) * in[i][b];
            out[i][a] = s;
        }
}

/* out = m in for a dense 4x4 spin matrix m */
static void spin_mat(const cplx m[4][4], const cplx *in, cplx *out)
{
    for (int i = 0; i < 4; i++)
        for (int c = 0; c < 3; c++) {
            cplx s = 0;
            for (int j = 0; j < 4; j++) s += m[i][j] * in[j * 3 + c];
            out[i * 3 + c] = s;
        }
}

/* the site term 1 + i * t * gamma_5 as a dense 4x4 matrix */
static void twist_matrix(double t, cplx m[4][4])
{
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) m[i][j] = (i == j ? 1.0 : 0.0) + I * t * GAMMA5[i][j];
}

/* ---------------------------------------------------------- operators */

/* out = H in over the full lattice (eq. (eo0) hopping term with the phase of Sec. 4.1.2) */
void orc_hop(const int *dims, const double *Ud, const double *theta, const double *ind, double *outd)
{
    init_gammas();
    geom g = make_geom(dims);
    const cplx *U = (const cplx *)Ud;
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    cplx ph[4];
    for (int mu = 0; mu < 4; mu++) ph[mu] = cexp(I * M_PI * theta[mu] / g.L[mu]);

#pragma omp parallel for schedule(static)
    for (long s = 0; s < g.V; s++) {
        cplx acc[4][3];
        memset(acc, 0, sizeof(acc));
        for (int mu = 0; mu < 4; mu++) {
            cplx v[4][3], w[4][3];
            long f = neighbour(&g, s, mu, +1);
            long b = neighbour(&g, s, mu, -1);
            /* forward: e^{i theta pi/L} U(x,mu) (1 + gamma_mu) psi(x+mu) */
            one_pm_gamma(mu, +1, in + 12 * f, v);
            colour_mul(U + (s * 4 + mu) * 9, 0, v, w);
            for (int i = 0; i < 4; i++)
                for (int c = 0; c < 3; c++) acc[i][c] += ph[mu] * w[i][c];
            /* backward: e^{-i theta pi/L} U(x-mu,mu)^+ (1 - gamma_mu) psi(x-mu) */
            one_pm_gamma(mu, -1, in + 12 * b, v);
            colour_mul(U + (b * 4 + mu) * 9, 1, v, w);
            for (int i = 0; i < 4; i++)
                for (int c = 0; c < 3; c++) acc[i][c] += conj(ph[mu]) * w[i][c];
        }
        for (int i = 0; i < 4; i++)
            for (int c = 0; c < 3; c++) out[s * 12 + i * 3 + c] = acc[i][c];
    }
}

/* out = M^{sign} in = (1 + sign i mut gamma_5) in - kappa H in  (full lattice) */
void orc_M(const int *dims, const double *U, double kappa, double mut, int sign,
           const double *theta, const double *ind, double *outd)
{
    init_gammas();
    geom g = make_geom(dims);
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    cplx tw[4][4];
    twist_matrix(sign * mut, tw);
    orc_hop(dims, U, theta, ind, outd);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g.V; s++) {
        cplx t[12];
        spin_mat(tw, in + 12 * s, t);
        for (int k = 0; k < 12; k++) out[12 * s + k] = t[k] - kappa * out[12 * s + k];
    }
}

/* out = Q^{sign} in = gamma_5 M^{sign} in (eq. (eo1)) */
void orc_Q(const int *dims, const double *U, double kappa, double mut, int sign,
           const double *theta, const double *ind, double *outd)
{
    geom g = make_geom(dims);
    cplx *out = (cplx *)outd;
    orc_M(dims, U, kappa, mut, sign, theta, ind, outd);
    for (long s = 0; s < g.V; s++) {
        cplx t[12];
        spin_mat(GAMMA5, out + 12 * s, t);
        memcpy(out + 12 * s, t, sizeof(t));
    }
}

/*
 * out_o = Qhat^{sign} in_o = gamma_5 [ M_oo in_o - M_oe (M_ee)^{-1} M_eo in_o ]
 * built literally: embed in_o in a full field, apply -kappa H, keep the even
 * part (M_eo in_o), apply (M_ee)^{-1} of eq. (eo3), embed, apply -kappa H,
 * keep the odd part, subtract from M_oo in_o and multiply by gamma_5.
 */
void orc_Qhat(const int *dims, const double *U, double kappa, double mut, int sign,
              const double *theta, const double *ind, double *outd)
{
    init_gammas();
    geom g = make_geom(dims);
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    long *odd = malloc(sizeof(long) * (g.V / 2));
    cplx *f1 = calloc((size_t)g.V * 12, sizeof(cplx));
    cplx *f2 = calloc((size_t)g.V * 12, sizeof(cplx));
    long nodd = orc_odd_sites(dims, odd);

    for (long k = 0; k < nodd; k++) memcpy(f1 + 12 * odd[k], in + 12 * k, 12 * sizeof(cplx));
    orc_hop(dims, U, theta, (const double *)f1, (double *)f2); /* f2 = H f1 */

    cplx mee_inv[4][4]; /* (1 - sign i mut g5) / (1 + mut^2) */
    twist_matrix(-sign * mut, mee_inv);
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) mee_inv[i][j] /= (1.0 + mut * mut);

    memset(f1, 0, (size_t)g.V * 12 * sizeof(cplx));
    for (long s = 0; s < g.V; s++) {
        if (parity(&g, s)) continue;
        cplx meo[12];
        for (int k = 0; k < 12; k++) meo[k] = -kappa * f2[12 * s + k]; /* M_eo in_o */
        spin_mat(mee_inv, meo, f1 + 12 * s);
    }
    orc_hop(dims, U, theta, (const double *)f1, (double *)f2); /* f2 = H f1 */

    cplx moo[4][4];
    twist_matrix(sign * mut, moo);
    for (long k = 0; k < nodd; k++) {
        cplx t[12], u[12];
        spin_mat(moo, in + 12 * k, t);
        for (int q = 0; q < 12; q++) t[q] -= -kappa * f2[12 * odd[k] + q]; /* - M_oe(...) */
        spin_mat(GAMMA5, t, u);
        memcpy(out + 12 * k, u, sizeof(u));
    }
    free(odd);
    free(f1);
    free(f2);
}

/* out = Qhat^+ Qhat^- in (Qhat^- applied first) */
void orc_QhatQhat(const int *dims, const double *U, double kappa, double mut,
                  const double *theta, const double *in, double *out)
{
    geom g = make_geom(dims);
    double *t = malloc(sizeof(cplx) * 12 * (size_t)(g.V / 2));
    orc_Qhat(dims, U, kappa, mut, -1, theta, in, t);
    orc_Qhat(dims, U, kappa, mut, +1, theta, t, out);
    free(t);
}

/* out = Q^+ Q^- in on the full lattice (Q^- applied first) */
void orc_QQ(const int *dims, const double *U, double kappa, double mut,
            const double *theta, const double *in, double *out)
{
    geom g = make_geom(dims);
    double *t = malloc(sizeof(cplx) * 12 * (size_t)g.V);
    orc_Q(dims, U, kappa, mut, -1, theta, in, t);
    orc_Q(dims, U, kappa, mut, +1, theta, t, out);
    free(t);
}

/* ----------------------------------------------------------------- CG */

static double dot_re(long n, const cplx *a, const cplx *b)
{
    double s = 0;
    for (long i = 0; i < n; i++) s += creal(conj(a[i]) * b[i]);
    return s;
}

typedef struct {
    const int *dims;
    const double *U;
    double kappa, mut;
    const double *theta;
    int eo;
} normal_op;

static void apply_normal(const normal_op *op, const cplx *in, cplx *out)
{
    if (op->eo)
        orc_QhatQhat(op->dims, op->U, op->kappa, op->mut, op->theta, (const double *)in, (double *)out);
    else
        orc_QQ(op->dims, op->U, op->kappa, op->mut, op->theta, (const double *)in, (double *)out);
}

/*
 * Textbook CG for A x = b with A = Qhat^+ Qhat^- (eo = 1, odd-site fields) or
 * A = Q^+ Q^- (eo = 0, full-lattice fields).  x_0 = 0.  Returns 0 when the
 * stopping criterion was met, 1 when max_iter was reached.  alpha/beta (may be
 * NULL, length max_iter) receive the CG coefficients, rr (may be NULL, length
 * max_iter + 1) the iterated ||r||^2 before each iteration and at the end.
 */
int orc_cg(const int *dims, const double *U, double kappa, double mut, const double *theta,
           int eo, const double *bd, double *xd, double tol, int relative, int max_iter,
           double *alpha, double *beta, double *rrhist, int *iters)
{
    geom g = make_geom(dims);
    long n = 12 * (eo ? g.V / 2 : g.V);
    const cplx *b = (const cplx *)bd;
    cplx *x = (cplx *)xd;
    cplx *r = malloc(sizeof(cplx) * n);
    cplx *p = malloc(sizeof(cplx) * n);
    cplx *Ap = malloc(sizeof(cplx) * n);
    normal_op op = {dims, U, kappa, mut, theta, eo};

    for (long i = 0; i < n; i++) {
        x[i] = 0;
        r[i] = b[i];
        p[i] = b[i];
    }
    double rr = dot_re(n, r, r);
    double target = relative ? tol * tol * rr : tol * tol;
    int k = 0, status = 1;
    for (;;) {
        if (rrhist) rrhist[k] = rr;
        if (rr < target || rr == 0.0) {
            status = 0;
            break;
        }
        if (k >= max_iter) break;
        apply_normal(&op, p, Ap);
        double a = rr / dot_re(n, p, Ap);
        for (long i = 0; i < n; i++) {
            x[i] += a * p[i];
            r[i] -= a * Ap[i];
        }
        double rr_new = dot_re(n, r, r);
        double bt = rr_new / rr;
        for (long i = 0; i < n; i++) p[i] = r[i] + bt * p[i];
        if (alpha) alpha[k] = a;
        if (beta) beta[k] = bt;
        rr = rr_new;
        k++;
    }
    *iters = k;
    free(r);
    free(p);
    free(Ap);
    return status;
}

/* ||b - A x|| / ||b|| with the same A as orc_cg (the true residual of Sec. 4.4) */
double orc_true_residual(const int *dims, const double *U, double kappa, double mut,
                         const double *theta, int eo, const double *bd, const double *xd)
{
    geom g = make_geom(dims);
    long n = 12 * (eo ? g.V / 2 : g.V);
    const cplx *b = (const cplx *)bd;
    cplx *Ax = malloc(sizeof(cplx) * n);
    normal_op op = {dims, U, kappa, mut, theta, eo};
    apply_normal(&op, (const cplx *)xd, Ax);
    double rr = 0, bb = 0;
    for (long i = 0; i < n; i++) {
        cplx d = b[i] - Ax[i];
        rr += creal(d * conj(d));
        bb += creal(b[i] * conj(b[i]));
    }
    free(Ax);
    return bb > 0 ? sqrt(rr / bb) : sqrt(rr);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * rkpm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the traditional (neighbour-loop)
 * Galerkin RKPM for the Poisson problem, written directly from the paper's
 * definitions.  It is the oracle the GPU path is checked against; only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header, table or constant generator with the GPU
 * library.
 *
 * What it computes (arXiv 2403.19854):
 *   - kernel: tensor-product cubic B-spline with rectangular support,
 *     a_k = at_k * h_k                                   (Sec 2.1, Eq 6, 7; Sec 5.1, Eq 64)
 *   - moment matrix M(x_S) = sum_J H(x_S-x_J) H^T(x_S-x_J) phi(x_S-x_J),
 *     summed over nodes J inside the domain (chi_J = 1)   (Sec 2.1, Eq 3; Sec 4.1, Eq 48)
 *   - shape functions Psi_J(x_S) = H^T(0) M^-1 H(x_S-x_J) phi   (Eq 2)
 *     and implicit gradients Psi^a_J = [H^grad_a]^T M^-1 H phi,
 *     H^grad_a = -e_{a+1}                                  (Sec 2.2, Eq 15, 16)
 *   - stiffness product with direct nodal integration:
 *     (K d)_I = sum_S V_S sum_a Psi^a_I(x_S) sum_J Psi^a_J(x_S) d_J
 *                                                          (Sec 2.3, Eq 26; Sec 4.2.2, Eq 54)
 *   - load f^r_I = sum_S V_S r_S Psi_I(x_S)                (Eq 27 with nodal quadrature, Eq 59)
 *   - field u^h_I = sum_J Psi_J(x_I) d_J                   (Sec 4.2.4, Eq 62)
 *   - linear CG on the rows/columns of the free nodes, strong Dirichlet values
 *                                                          (Sec 2.4, Eq 29; Sec 5.4.3)
 *
 * Neighbour lookups are NOT periodic: an index outside [0, n_k) does not exist.
 * This is the "traditional RKPM on the nodes of Omega, no extension" the paper
 * compares against (Sec 6.1.1).
 *
 * Basis: graded-lex monomials of the offsets scaled by h (z_k / h_k).  A
 * linear change of basis leaves Psi unchanged; it rescales the implicit
 * gradient vectors by 1/h_k, which is applied explicitly below.
 *
 * Layout: node index I = x + n0*(y + n1*z), x fastest.  All arrays FP64 except
 * the 0/1 masks (uint8).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXS 35

typedef struct {
    int dim;
    int n[3];
    long nn;
    double h[3];
    double at[3];
    int m[3];
    int degree;
    int s;
    int ex[ORC_MAXS][3];
    uint8_t *chi;
    double *vol;
    int noff;
    int *off;        /* noff x 3 integer offsets o (J = S + o)            */
    double *phiw;    /* phi((x_S - x_J)) = phi(-o h), noff                */
    double *hm;      /* H~(-o), noff x s                                   */
    double *b0;      /* nn x s          (zero where chi = 0)              */
    double *ba;      /* nn x dim x s    (zero where chi = 0)              */
    long singular_node;
} orc_ctx;

/* Cubic B-spline profile, Eq 7, z = |x| / a. */
double orc_phi1(double z)
{
    z = fabs(z);
    if (z <= 0.5) return 2.0 / 3.0 - 4.0 * z * z + 4.0 * z * z * z;
    if (z < 1.0) return 4.0 / 3.0 - 4.0 * z + 4.0 * z * z - 4.0 / 3.0 * z * z * z;
    return 0.0; /* the second piece vanishes at z = 1 */
}

static double ipow(double x, int e)
{
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

/* Graded-lex exponents of the monomials of degree <= n in d variables
 * (Eq 4 gives the 2D order 1, x, y, x^2, xy, y^2). */
static int make_basis(int dim, int degree, int ex[ORC_MAXS][3])
{
    int s = 0;
    for (int deg = 0; deg <= degree; ++deg) {
        for (int ax = deg; ax >= 0; --ax) {
            if (dim == 1) {
                if (ax != deg) continue;
                ex[s][0] = ax; ex[s][1] = 0; ex[s][2] = 0; ++s;
                continue;
            }
            for (int ay = deg - ax; ay >= 0; --ay) {
                int az = deg - ax - ay;
                if (dim == 2 && az != 0) continue;
                ex[s][0] = ax; ex[s][1] = ay; ex[s][2] = az; ++s;
            }
        }
    }
    return s;
}

/* Threads of the parallel loops below: n > 0 sets them, any n returns the
 * count in force afterwards (timing plumbing; no arithmetic depends on it). */
int orc_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}

int orc_basis_size(int dim, int degree)
{
    int ex[ORC_MAXS][3];
    return make_basis(dim, degree, ex);
}

static void coords(const orc_ctx *c, long I, int *i)
{
    i[0] = (int)(I % c->n[0]);
    i[1] = (int)((I / c->n[0]) % c->n[1]);
    i[2] = (int)(I / ((long)c->n[0] * c->n[1]));
}

/* J = S + o if inside the box (non-periodic), else -1. */
static long shift(const orc_ctx *c, const int *i, const int *o)
{
    int j[3];
    for (int k = 0; k < 3; ++k) {
        j[k] = i[k] + o[k];
        if (j[k] < 0 || j[k] >= c->n[k]) return -1;
    }
    return (long)j[0] + (long)c->n[0] * ((long)j[1] + (long)c->n[1] * j[2]);
}

/* Cholesky of the s x s SPD matrix a (row-major, lower part used) in place.
 * Returns 0 on success, -1 if a pivot is <= tol. */
static int cholesky(double *a, int s, double tol)
{
    for (int j = 0; j < s; ++j) {
        double d = a[j * s + j];
        for (int k = 0; k < j; ++k) d -= a[j * s + k] * a[j * s + k];
        if (!(d > tol)) return -1;
        d = sqrt(d);
        a[j * s + j] = d;
        for (int i = j + 1; i < s; ++i) {
            double v = a[i * s + j];
            for (int k = 0; k < j; ++k) v -= a[i * s + k] * a[j * s + k];
            a[i * s + j] = v / d;
        }
    }
    return 0;
}

/* Solve L L^T y = e_col. */
static void chol_solve_unit(const double *l, int s, int col, double *y)
{
    double z[ORC_MAXS];
    for (int i = 0; i < s; ++i) {
        double v = (i == col) ? 1.0 : 0.0;
        for (int k = 0; k < i; ++k) v -= l[i * s + k] * z[k];
        z[i] = v / l[i * s + i];
    }
    for (int i = s - 1; i >= 0; --i) {
        double v = z[i];
        for (int k = i + 1; k < s; ++k) v -= l[k * s + i] * y[k];
        y[i] = v / l[i * s + i];
    }
}

void orc_destroy(orc_ctx *c)
{
    if (!c) return;
    free(c->chi); free(c->vol); free(c->off); free(c->phiw); free(c->hm);
    free(c->b0); free(c->ba);
    free(c);
}

long orc_singular_node(const orc_ctx *c) { return c->singular_node; }
int orc_s(const orc_ctx *c) { return c->s; }
int orc_noff(const orc_ctx *c) { return c->noff; }

/*
 * Build the context: neighbour offsets, per-node moment matrices (Eq 3 over
 * domain nodes), their Cholesky factors and the rows of M^-1 that give b^0
 * (Eq 45, 83) and the implicit-gradient vectors b^a (Eq 46-47, 84-85).
 * vol may be NULL (then V = prod h on every domain node).
 * Returns NULL on allocation failure; sets singular_node >= 0 if some M is
 * not SPD (pivot <= 1e-13 * trace).
 */
orc_ctx *orc_create(int dim, const int *n, const double *h, const double *at,
                    int degree, const uint8_t *chi, const double *vol)
{
    orc_ctx *c = (orc_ctx *)calloc(1, sizeof(orc_ctx));
    if (!c) return NULL;
    c->dim = dim;
    c->degree = degree;
    for (int k = 0; k < 3; ++k) {
        c->n[k] = (k < dim) ? n[k] : 1;
        c->h[k] = (k < dim) ? h[k] : 1.0;
        c->at[k] = (k < dim) ? at[k] : 0.0;
        c->m[k] = (k < dim) ? (int)floor(at[k]) : 0;
    }
    c->nn = (long)c->n[0] * c->n[1] * c->n[2];
    c->s = make_basis(dim, degree, c->ex);
    c->singular_node = -1;

    c->chi = (uint8_t *)malloc(c->nn);
    c->vol = (double *)malloc(sizeof(double) * c->nn);
    if (!c->chi || !c->vol) { orc_destroy(c); return NULL; }
    memcpy(c->chi, chi, c->nn);
    double hv = c->h[0] * c->h[1] * c->h[2];
    for (long I = 0; I < c->nn; ++I)
        c->vol[I] = vol ? vol[I] : (chi[I] ? hv : 0.0);

    /* offsets o with |o_k| <= floor(at_k) and non-zero kernel weight */
    int cnt = (2 * c->m[0] + 1) * (2 * c->m[1] + 1) * (2 * c->m[2] + 1);
    c->off = (int *)malloc(sizeof(int) * 3 * cnt);
    c->phiw = (double *)malloc(sizeof(double) * cnt);
    c->hm = (double *)malloc(sizeof(double) * cnt * c->s);
    if (!c->off || !c->phiw || !c->hm) { orc_destroy(c); return NULL; }
    int q = 0;
    for (int oz = -c->m[2]; oz <= c->m[2]; ++oz)
        for (int oy = -c->m[1]; oy <= c->m[1]; ++oy)
            for (int ox = -c->m[0]; ox <= c->m[0]; ++ox) {
                int o[3] = {ox, oy, oz};
                /* x_S - x_J = -o h, and |x_k| / a_k = |o_k| h_k / (at_k h_k) */
                double w = 1.0;
                for (int k = 0; k < dim; ++k)
                    w *= orc_phi1((double)abs(o[k]) / c->at[k]);
                if (w == 0.0) continue;
                c->off[3 * q + 0] = ox; c->off[3 * q + 1] = oy; c->off[3 * q + 2] = oz;
                c->phiw[q] = w;
                for (int p = 0; p < c->s; ++p) {
                    double v = 1.0;
                    for (int k = 0; k < dim; ++k) v *= ipow((double)(-o[k]), c->ex[p][k]);
                    c->hm[q * c->s + p] = v;
                }
                ++q;
            }
    c->noff = q;

    int s = c->s;
    c->b0 = (double *)calloc((size_t)c->nn * s, sizeof(double));
    c->ba = (double *)calloc((size_t)c->nn * dim * s, sizeof(double));
    if (!c->b0 || !c->ba) { orc_destroy(c); return NULL; }

    long bad = -1;
#pragma omp parallel for schedule(dynamic, 256) reduction(max : bad)
    for (long S = 0; S < c->nn; ++S) {
        if (!c->chi[S]) continue;
        int i[3];
        coords(c, S, i);
        double M[ORC_MAXS * ORC_MAXS];
        memset(M, 0, sizeof(double) * s * s);
        for (int t = 0; t < c->noff; ++t) {
            long J = shift(c, i, &c->off[3 * t]);
            if (J < 0 || !c->chi[J]) continue;
            const double *v = &c->hm[t * s];
            double w = c->phiw[t];
            for (int a = 0; a < s; ++a)
                for (int b = 0; b < s; ++b) M[a * s + b] += v[a] * v[b] * w;
        }
        double tr = 0.0;
        for (int a = 0; a < s; ++a) tr += M[a * s + a];
        if (cholesky(M, s, 1e-13 * tr) != 0) {
            /* record the largest failing index; the caller only needs one */
            if (S > bad) bad = S;
            continue;
        }
        double y[ORC_MAXS];
        chol_solve_unit(M, s, 0, y);
        for (int p = 0; p < s; ++p) c->b0[S * s + p] = y[p];
        for (int a = 0; a < dim; ++a) {
            chol_solve_unit(M, s, 1 + a, y);
            for (int p = 0; p < s; ++p)
                c->ba[(S * dim + a) * s + p] = -y[p] / c->h[a];
        }
    }
    c->singular_node = bad;
    return c;
}

void orc_get_b0(const orc_ctx *c, double *out)
{
    memcpy(out, c->b0, sizeof(double) * c->nn * c->s);
}

void orc_get_ba(const orc_ctx *c, double *out)
{
    memcpy(out, c->ba, sizeof(double) * c->nn * c->dim * c->s);
}

/* Psi-type weight of node J = S + o evaluated at x_S with coefficient vector b
 * of node S: b . H~(-o) phi(-o h). */
static inline double shape_w(const orc_ctx *c, const double *b, int t)
{
    const double *v = &c->hm[t * c->s];
    double acc = 0.0;
    for (int p = 0; p < c->s; ++p) acc += b[p] * v[p];
    return acc * c->phiw[t];
}

/* Implicit-gradient field g^a_S = sum_J Psi^a_J(x_S) d_J at every domain node
 * (B d, Eq 19 with Eq 15).  g is dim x nn. */
void orc_apply_b(const orc_ctx *c, const double *d, double *g)
{
    int dim = c->dim, s = c->s;
#pragma omp parallel for schedule(static)
    for (long S = 0; S < c->nn; ++S) {
        double acc[3] = {0.0, 0.0, 0.0};
        if (c->chi[S]) {
            int i[3];
            coords(c, S, i);
            for (int t = 0; t < c->noff; ++t) {
                long J = shift(c, i, &c->off[3 * t]);
                if (J < 0 || !c->chi[J]) continue;
                for (int a = 0; a < dim; ++a)
                    acc[a] += shape_w(c, &c->ba[(S * dim + a) * s], t) * d[J];
            }
        }
        for (int a = 0; a < dim; ++a) g[a * c->nn + S] = acc[a];
    }
}

/* Transpose of the gradient operator with quadrature weights:
 * f_I = sum_S V_S sum_a Psi^a_I(x_S) g^a_S, restricted to domain nodes I. */
static void apply_bt_v(const orc_ctx *c, const double *g, double *f)
{
    int dim = c->dim, s = c->s;
#pragma omp parallel for schedule(static)
    for (long I = 0; I < c->nn; ++I) {
        double acc = 0.0;
        if (c->chi[I]) {
            int i[3];
            coords(c, I, i);
            for (int t = 0; t < c->noff; ++t) {
                /* S = I - o, so that I = S + o */
                int mo[3] = {-c->off[3 * t], -c->off[3 * t + 1], -c->off[3 * t + 2]};
                long S = shift(c, i, mo);
                if (S < 0 || !c->chi[S]) continue;
                double w = 0.0;
                for (int a = 0; a < dim; ++a)
                    w += shape_w(c, &c->ba[(S * dim + a) * s], t) * g[a * c->nn + S];
                acc += c->vol[S] * w;
            }
        }
        f[I] = acc;
    }
}

/* B^T (V o g) for a dim x nn field g (the force of a gradient nonlinearity,
 * Eq B.6-B.8). */
void orc_apply_btv(const orc_ctx *c, const double *g, double *f) { apply_bt_v(c, g, f); }

/* Unmasked stiffness product f = K d over all domain nodes (Eq 26, Eq 54). */
void orc_apply_k(const orc_ctx *c, const double *d, double *f)
{
    double *g = (double *)malloc(sizeof(double) * c->nn * c->dim);
    orc_apply_b(c, d, g);
    apply_bt_v(c, g, f);
    free(g);
}

/* (K d)_I at the listed nodes only; g^a is recomputed locally per neighbour.
 * For spot checks on large grids. */
void orc_apply_k_at(const orc_ctx *c, const double *d, const long *idx, long nidx, double *f)
{
    int dim = c->dim, s = c->s;
#pragma omp parallel for schedule(dynamic, 1)
    for (long q = 0; q < nidx; ++q) {
        long I = idx[q];
        double acc = 0.0;
        if (c->chi[I]) {
            int i[3];
            coords(c, I, i);
            for (int t = 0; t < c->noff; ++t) {
                int mo[3] = {-c->off[3 * t], -c->off[3 * t + 1], -c->off[3 * t + 2]};
                long S = shift(c, i, mo);
                if (S < 0 || !c->chi[S]) continue;
                int si[3];
                coords(c, S, si);
                double g[3] = {0.0, 0.0, 0.0};
                for (int u = 0; u < c->noff; ++u) {
                    long J = shift(c, si, &c->off[3 * u]);
                    if (J < 0 || !c->chi[J]) continue;
                    for (int a = 0; a < dim; ++a)
                        g[a] += shape_w(c, &c->ba[(S * dim + a) * s], u) * d[J];
                }
                double w = 0.0;
                for (int a = 0; a < dim; ++a)
                    w += shape_w(c, &c->ba[(S * dim + a) * s], t) * g[a];
                acc += c->vol[S] * w;
            }
        }
        f[q] = acc;
    }
}

/* y -> N^T (w o y):  f_I = sum_S w_S y_S Psi_I(x_S)  on domain nodes.
 * With w = V this is the load vector f^r (Eq 59); with w = 1 it is N^T y. */
static void apply_nt_w(const orc_ctx *c, const double *y, const double *w, double *f)
{
    int s = c->s;
#pragma omp parallel for schedule(static)
    for (long I = 0; I < c->nn; ++I) {
        double acc = 0.0;
        if (c->chi[I]) {
            int i[3];
            coords(c, I, i);
            for (int t = 0; t < c->noff; ++t) {
                int mo[3] = {-c->off[3 * t], -c->off[3 * t + 1], -c->off[3 * t + 2]};
                long S = shift(c, i, mo);
                if (S < 0 || !c->chi[S]) continue;
                double ws = w ? w[S] : 1.0;
                acc += ws * y[S] * shape_w(c, &c->b0[S * s], t);
            }
        }
        f[I] = acc;
    }
}

void orc_apply_fr(const orc_ctx *c, const double *r, double *f) { apply_nt_w(c, r, c->vol, f); }
void orc_apply_nt(const orc_ctx *c, const double *y, double *f) { apply_nt_w(c, y, NULL, f); }

/* u^h_I = sum_J Psi_J(x_I) d_J on domain nodes (Eq 62). */
void orc_apply_uh(const orc_ctx *c, const double *d, double *u)
{
    int s = c->s;
#pragma omp parallel for schedule(static)
    for (long I = 0; I < c->nn; ++I) {
        double acc = 0.0;
        if (c->chi[I]) {
            int i[3];
            coords(c, I, i);
            for (int t = 0; t < c->noff; ++t) {
                long J = shift(c, i, &c->off[3 * t]);
                if (J < 0 || !c->chi[J]) continue;
                acc += shape_w(c, &c->b0[I * s], t) * d[J];
            }
        }
        u[I] = acc;
    }
}

/* V o (N z) */
void orc_apply_vn(const orc_ctx *c, const double *z, double *out)
{
    orc_apply_uh(c, z, out);
    for (long I = 0; I < c->nn; ++I) out[I] *= c->vol[I];
}

static double dot(const double *a, const double *b, long n)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/*
 * Linear CG on the free rows/columns (mask free[] = chi_Omega, Eq 96):
 * solves K_ff x_f = rhs_f starting from the x given (x outside free nodes is
 * ignored and left at zero in the product).  Stops when ||r||_2 / ||rhs||_2 <= tol
 * on the recursive residual, or after maxit iterations.
 * Returns the iteration count; *relres receives the final recursive residual.
 */
int orc_cg(const orc_ctx *c, const uint8_t *free_, const double *rhs, double *x,
           double tol, int maxit, double *relres)
{
    long nn = c->nn;
    double *r = (double *)malloc(sizeof(double) * nn);
    double *p = (double *)malloc(sizeof(double) * nn);
    double *q = (double *)malloc(sizeof(double) * nn);
    double *xm = (double *)malloc(sizeof(double) * nn);
    for (long i = 0; i < nn; ++i) xm[i] = free_[i] ? x[i] : 0.0;
    orc_apply_k(c, xm, q);
    for (long i = 0; i < nn; ++i) {
        r[i] = free_[i] ? rhs[i] - q[i] : 0.0;
        p[i] = r[i];
        x[i] = xm[i];
    }
    double bb = 0.0;
    for (long i = 0; i < nn; ++i) if (free_[i]) bb += rhs[i] * rhs[i];
    double bn = sqrt(bb);
    double rr = dot(r, r, nn);
    int it = 0;
    if (bn == 0.0) bn = 1.0;
    while (it < maxit && sqrt(rr) / bn > tol) {
        orc_apply_k(c, p, q);
        for (long i = 0; i < nn; ++i) if (!free_[i]) q[i] = 0.0;
        double pq = dot(p, q, nn);
        if (!(pq > 0.0)) break;
        double alpha = rr / pq;
        for (long i = 0; i < nn; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        double rr2 = dot(r, r, nn);
        double beta = rr2 / rr;
        for (long i = 0; i < nn; ++i) p[i] = r[i] + beta * p[i];
        rr = rr2;
        ++it;
    }
    if (relres) *relres = sqrt(rr) / bn;
    free(r); free(p); free(q); free(xm);
    return it;
}

/*
 * Static solve (Sec 5.4.3, Alg 5 outline): d = g on Dirichlet nodes (Eq 29),
 * f^r from r, rhs = chi_Omega o (f^r - K d_Gamma), CG from d_Omega = x (in/out:
 * pass zeros for the paper's start).  g may be NULL (homogeneous).
 */
int orc_solve(const orc_ctx *c, const uint8_t *free_, const uint8_t *dir,
              const double *r, const double *g, double *d, double tol, int maxit,
              double *relres)
{
    long nn = c->nn;
    double *fr = (double *)malloc(sizeof(double) * nn);
    double *dg = (double *)calloc(nn, sizeof(double));
    double *kg = (double *)malloc(sizeof(double) * nn);
    orc_apply_fr(c, r, fr);
    if (g && dir)
        for (long i = 0; i < nn; ++i) if (dir[i]) dg[i] = g[i];
    orc_apply_k(c, dg, kg);
    for (long i = 0; i < nn; ++i) fr[i] = free_[i] ? fr[i] - kg[i] : 0.0;
    int it = orc_cg(c, free_, fr, d, tol, maxit, relres);
    for (long i = 0; i < nn; ++i) if (dir && dir[i]) d[i] = dg[i];
    free(fr); free(dg); free(kg);
    return it;
}

/*
 * Adjoint of u^h(r) = N d(r), d solving the homogeneous strong-Dirichlet
 * problem:  dL/dr = V o N z,  z = K_ff^-1 chi_Omega o N^T(dL/du^h).
 * z is returned as well (may be NULL).
 */
int orc_adjoint(const orc_ctx *c, const uint8_t *free_, const double *dl_du,
                double *dl_dr, double *z_out, double tol, int maxit, double *relres)
{
    long nn = c->nn;
    double *y = (double *)malloc(sizeof(double) * nn);
    double *z = (double *)calloc(nn, sizeof(double));
    orc_apply_nt(c, dl_du, y);
    for (long i = 0; i < nn; ++i) if (!free_[i]) y[i] = 0.0;
    int it = orc_cg(c, free_, y, z, tol, maxit, relres);
    orc_apply_vn(c, z, dl_dr);
    if (z_out) memcpy(z_out, z, sizeof(double) * nn);
    free(y); free(z);
    return it;
}

/*
 * Oracle for the FMM-accelerated BEM mat-vec and its GMRES solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, FP64 CPU code written from the paper
 * (Wang, Layton & Barba, "Inexact Krylov iterations and relaxation strategies
 * with fast-multipole boundary element method").  Only the tests, the smoke
 * check and the bench's CPU-baseline leg may load it; the product path never
 * does, and this file shares no code, header or table with it.
 *
 * What it computes is the dense collocation matrix that the FMM approximates:
 *   - constant flat triangular panels, collocation at centroids (Sec. 2.1, Eq. 2-3);
 *   - Laplace single layer, G = 1/(4 pi r) (Sec. 2.1, Eq. 4); the 1/(4 pi) is kept;
 *   - Stokes single layer, u = -1/(8 pi mu) sum_J t_J int G (Sec. 2.2, Eq. 6, 7, 9);
 *   - Laplace double layer, second kind (Sec. 2.1, Eq. 5 and 11): with outward
 *     unit normals, the exterior Neumann problem (1/2 I - K) u = -V du/dn,
 *     K u = sum_j u_j int_j dG/dn_y, dG/dn_y = n_j . (x - y) / (4 pi |x - y|^3);
 *   - far panels: a K=4 Gauss rule, weights q_k S_j (Sec. 2.3, Eq. 10);
 *   - near-singular panels, within 2 sqrt(2 S_j) of the target (Sec. 2.3,
 *     figure on integration domains): a 25-point collapsed Gauss-Legendre rule;
 *   - the panel holding the target: the radial part of the polar split about
 *     the target (Hess-Smith decomposition, Sec. 2.3) integrated exactly, and
 *     here also the angular part, in closed form;
 *   - the mat-vec as the sum over targets of sources (Eq. 12, Appendix A,
 *     matrix-vector multiplication algorithm);
 *   - GMRES(m) with modified Gram-Schmidt and Givens rotations (Sec. 2.4), no
 *     expansion order and no FMM.
 * Readings where the paper is silent (which 4-point rule, which near rule, the
 * distance in the near test, the restart) are stated beside the code.
 * Compiled with -ffp-contract=off so that every product and sum is rounded as
 * written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* Panel geometry (Sec. 2.1): centroid, area S = |a|/2 and unit normal a/|a|, */
/* a = (v1 - v0) x (v2 - v0).                                               */
/* ------------------------------------------------------------------------- */
static void panel_geom(const double *v0, const double *v1, const double *v2,
                       double *c, double *S, double *n)
{
    double e1[3], e2[3], a[3];
    for (int d = 0; d < 3; ++d) {
        c[d] = ((v0[d] + v1[d]) + v2[d]) / 3.0;
        e1[d] = v1[d] - v0[d];
        e2[d] = v2[d] - v0[d];
    }
    a[0] = e1[1] * e2[2] - e1[2] * e2[1];
    a[1] = e1[2] * e2[0] - e1[0] * e2[2];
    a[2] = e1[0] * e2[1] - e1[1] * e2[0];
    double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    *S = 0.5 * na;
    if (n) {
        for (int d = 0; d < 3; ++d)
            n[d] = a[d] / na;
    }
}

void or_panels(int64_t nt, const double *xyz, const int32_t *tri,
               double *c, double *S, double *nrm)
{
    for (int64_t j = 0; j < nt; ++j) {
        const int32_t *t = tri + 3 * j;
        panel_geom(xyz + 3 * (int64_t)t[0], xyz + 3 * (int64_t)t[1], xyz + 3 * (int64_t)t[2],
                   c + 3 * j, S + j, nrm ? nrm + 3 * j : NULL);
    }
}

/* ------------------------------------------------------------------------- */
/* Quadrature rules on the triangle, barycentric points and area-normalised   */
/* weights q_k (sum q_k = 1), as in Eq. (10).                                 */
/* ------------------------------------------------------------------------- */

/* Far rule, K = 4 (Sec. 2.3).  The paper does not name it; the reading is the
 * degree-3 rule with the centroid (weight -27/48) and the three permutations of
 * (0.6, 0.2, 0.2) (weight 25/48 each). */
int or_far_rule(double *bary, double *w)
{
    const double a = 1.0 / 3.0;
    double pts[4][3] = {{a, a, a}, {0.6, 0.2, 0.2}, {0.2, 0.6, 0.2}, {0.2, 0.2, 0.6}};
    double ww[4] = {-27.0 / 48.0, 25.0 / 48.0, 25.0 / 48.0, 25.0 / 48.0};
    for (int k = 0; k < 4; ++k) {
        for (int d = 0; d < 3; ++d)
            bary[3 * k + d] = pts[k][d];
        w[k] = ww[k];
    }
    return 4;
}

/* Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on P_n,
 * P_n from the three-term recurrence, w = 2 / ((1 - x^2) P_n'(x)^2).
 * Nodes in ascending order. */
void or_gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        /* root i counted from +1 downwards */
        double z = cos(OR_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) {
                p0 = 1.0;
                p1 = z;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16)
                break;
        }
        /* final derivative at the converged root */
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[n - 1 - i] = z;
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* Near-singular rule (Sec. 2.3 asks for K about 20; the reading is 25 points):
 * an n1d x n1d Gauss-Legendre product rule on the unit square, collapsed onto
 * the triangle, lambda = (1 - s, s (1 - t), s t), weight 2 s w_s w_t with w_s,
 * w_t the [0,1] weights.  Returns the number of points. */
int or_near_rule(int n1d, double *bary, double *w)
{
    double x[64], wx[64];
    if (n1d < 1 || n1d > 64)
        return 0;
    or_gauss_legendre(n1d, x, wx);
    int k = 0;
    for (int a = 0; a < n1d; ++a) {
        double s = 0.5 * (x[a] + 1.0), ws = 0.5 * wx[a];
        for (int b = 0; b < n1d; ++b) {
            double t = 0.5 * (x[b] + 1.0), wt = 0.5 * wx[b];
            bary[3 * k + 0] = 1.0 - s;
            bary[3 * k + 1] = s * (1.0 - t);
            bary[3 * k + 2] = s * t;
            w[k] = 2.0 * s * ws * wt;
            ++k;
        }
    }
    return k;
}

static void bary_point(const double *v0, const double *v1, const double *v2,
                       const double *l, double *y)
{
    for (int d = 0; d < 3; ++d)
        y[d] = (l[0] * v0[d] + l[1] * v1[d]) + l[2] * v2[d];
}

/* ------------------------------------------------------------------------- */
/* Integrals over the panel that holds the target (Sec. 2.3).               */
/* The target x lies in the panel's plane, inside the triangle (it is the   */
/* centroid).  In polar coordinates about x the radial integral of 1/r * r   */
/* is the distance R(phi) to the boundary; for an edge at perpendicular      */
/* distance h, R = h / cos(theta) with theta measured from the foot of the   */
/* perpendicular, and                                                        */
/*   int h / cos(theta) dtheta            = h asinh(tan theta)               */
/*   int h cos(theta)^2 / cos(theta)      = h sin(theta)                     */
/*   int h sin(theta)^2 / cos(theta)      = h (asinh(tan theta) - sin theta) */
/*   int h sin(theta) cos(theta)/cos(theta) = -h cos(theta)                  */
/* which give int 1/r dA and J = int e e^T / r dA (e the in-plane unit       */
/* vector from x) in closed form, edge by edge.                              */
/* ------------------------------------------------------------------------- */
static void self_integrals(const double *v0, const double *v1, const double *v2,
                           const double *x, double *I, double *J /* 3x3 or NULL */)
{
    const double *V[3] = {v0, v1, v2};
    double sumI = 0.0;
    double sJ[9] = {0};
    for (int e = 0; e < 3; ++e) {
        const double *a = V[e], *b = V[(e + 1) % 3];
        double ev[3], ax[3];
        for (int d = 0; d < 3; ++d) {
            ev[d] = b[d] - a[d];
            ax[d] = a[d] - x[d];
        }
        double L = sqrt(ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2]);
        double v[3] = {ev[0] / L, ev[1] / L, ev[2] / L};
        double sa = ax[0] * v[0] + ax[1] * v[1] + ax[2] * v[2]; /* along-edge coord of a */
        double sb = sa + L;
        double u[3] = {ax[0] - sa * v[0], ax[1] - sa * v[1], ax[2] - sa * v[2]}; /* foot - x */
        double h = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        for (int d = 0; d < 3; ++d)
            u[d] /= h;
        double ta = sa / h, tb = sb / h;
        double Ia = asinh(ta), Ib = asinh(tb);
        sumI += h * (Ib - Ia);
        if (J) {
            double ra = sqrt(sa * sa + h * h), rb = sqrt(sb * sb + h * h);
            double sin_a = sa / ra, sin_b = sb / rb, cos_a = h / ra, cos_b = h / rb;
            double cuu = h * (sin_b - sin_a);
            double cvv = h * ((Ib - sin_b) - (Ia - sin_a));
            double cuv = -h * (cos_b - cos_a);
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q)
                    sJ[3 * p + q] += cuu * u[p] * u[q] + cvv * v[p] * v[q] +
                                     cuv * (u[p] * v[q] + v[p] * u[q]);
        }
    }
    *I = sumI;
    if (J)
        memcpy(J, sJ, sizeof(sJ));
}

double or_laplace_self(const double *v0, const double *v1, const double *v2, const double *x)
{
    double I;
    self_integrals(v0, v1, v2, x, &I, NULL);
    return I;
}

void or_stokes_self(const double *v0, const double *v1, const double *v2, const double *x,
                    double *I, double *J)
{
    self_integrals(v0, v1, v2, x, I, J);
}

/* ------------------------------------------------------------------------- */
/* Dense mat-vec (Eq. 12; Appendix A).                                       */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t nt;
    const double *xyz;
    const int32_t *tri;
    double *c, *S, *n;      /* centroids, areas, unit normals */
    double fb[12], fw[4];   /* far rule */
    double nb[75], nw[25];  /* near rule */
    int nfar, nnear;
} mesh_t;

static int mesh_init(mesh_t *m, int64_t nt, const double *xyz, const int32_t *tri)
{
    m->nt = nt;
    m->xyz = xyz;
    m->tri = tri;
    m->c = (double *)malloc(sizeof(double) * 3 * (size_t)nt);
    m->S = (double *)malloc(sizeof(double) * (size_t)nt);
    m->n = (double *)malloc(sizeof(double) * 3 * (size_t)nt);
    if (!m->c || !m->S || !m->n)
        return -1;
    or_panels(nt, xyz, tri, m->c, m->S, m->n);
    m->nfar = or_far_rule(m->fb, m->fw);
    m->nnear = or_near_rule(5, m->nb, m->nw);
    return 0;
}

static void mesh_free(mesh_t *m)
{
    free(m->c);
    free(m->S);
    free(m->n);
}

#define VTX(m, j, a) ((m)->xyz + 3 * (int64_t)(m)->tri[3 * (j) + (a)])

/* Classification of (target i, source panel j), Sec. 2.3: the panel itself,
 * near-singular when the squared distance between the target and the source
 * panel's centroid is below 8 S_j (distance below 2 sqrt(2 S_j)), far else. */
static int classify(const mesh_t *m, int64_t i, int64_t j)
{
    if (i == j)
        return 2;
    double dx = m->c[3 * i] - m->c[3 * j];
    double dy = m->c[3 * i + 1] - m->c[3 * j + 1];
    double dz = m->c[3 * i + 2] - m->c[3 * j + 2];
    double d2 = (dx * dx + dy * dy) + dz * dz;
    return d2 < 8.0 * m->S[j] ? 1 : 0;
}

/* int_{panel j} 1/|x - y| dA by the rule for its class */
static double laplace_entry(const mesh_t *m, int64_t i, int64_t j)
{
    const double *v0 = VTX(m, j, 0), *v1 = VTX(m, j, 1), *v2 = VTX(m, j, 2);
    const double *x = m->c + 3 * i;
    int cls = classify(m, i, j);
    if (cls == 2)
        return or_laplace_self(v0, v1, v2, x);
    const double *B = cls ? m->nb : m->fb, *W = cls ? m->nw : m->fw;
    int np = cls ? m->nnear : m->nfar;
    double acc = 0.0;
    for (int k = 0; k < np; ++k) {
        double y[3];
        bary_point(v0, v1, v2, B + 3 * k, y);
        double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
        double r = sqrt((dx * dx + dy * dy) + dz * dz);
        acc += W[k] * m->S[j] / r;
    }
    return acc;
}

/* int_{panel j} n_j . (x - y) / |x - y|^3 dA (Eq. 11 without 1/(4 pi)) by the rule
 * for its class.  On the target's own flat panel x and every y lie in one plane,
 * n_j . (x - y) = 0, so the principal value is 0 (the 1/2 of the jump is the
 * identity term of the operator). */
static double dl_entry(const mesh_t *m, int64_t i, int64_t j)
{
    int cls = classify(m, i, j);
    if (cls == 2)
        return 0.0;
    const double *v0 = VTX(m, j, 0), *v1 = VTX(m, j, 1), *v2 = VTX(m, j, 2);
    const double *x = m->c + 3 * i, *nj = m->n + 3 * j;
    const double *B = cls ? m->nb : m->fb, *W = cls ? m->nw : m->fw;
    int np = cls ? m->nnear : m->nfar;
    double acc = 0.0;
    for (int k = 0; k < np; ++k) {
        double y[3];
        bary_point(v0, v1, v2, B + 3 * k, y);
        double d[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
        double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
        double r = sqrt(r2);
        double nd = (nj[0] * d[0] + nj[1] * d[1]) + nj[2] * d[2];
        acc += W[k] * m->S[j] * nd / (r2 * r);
    }
    return acc;
}

/* 3x3 block int_{panel j} G(x, y) dA, G_ab = delta_ab / r + d_a d_b / r^3, d = x - y (Eq. 7) */
static void stokes_entry(const mesh_t *m, int64_t i, int64_t j, double *G)
{
    const double *v0 = VTX(m, j, 0), *v1 = VTX(m, j, 1), *v2 = VTX(m, j, 2);
    const double *x = m->c + 3 * i;
    int cls = classify(m, i, j);
    if (cls == 2) {
        double I, J[9];
        or_stokes_self(v0, v1, v2, x, &I, J);
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q)
                G[3 * p + q] = (p == q ? I : 0.0) + J[3 * p + q];
        return;
    }
    const double *B = cls ? m->nb : m->fb, *W = cls ? m->nw : m->fw;
    int np = cls ? m->nnear : m->nfar;
    for (int p = 0; p < 9; ++p)
        G[p] = 0.0;
    for (int k = 0; k < np; ++k) {
        double y[3];
        bary_point(v0, v1, v2, B + 3 * k, y);
        double d[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
        double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
        double r = sqrt(r2);
        double wk = W[k] * m->S[j];
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q)
                G[3 * p + q] += wk * ((p == q ? 1.0 / r : 0.0) + d[p] * d[q] / (r2 * r));
    }
}

/* y = A x for the Laplace single layer, A_ij = (1/4pi) int_j 1/r.  When
 * `rows` is non-NULL only those nrows rows are computed, into y[0..nrows). */
int or_matvec_laplace(int64_t nt, const double *xyz, const int32_t *tri,
                      const double *x, double *y, int64_t nrows, const int64_t *rows)
{
    mesh_t m;
    if (mesh_init(&m, nt, xyz, tri))
        return -1;
    int64_t nr = rows ? nrows : nt;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nr; ++r) {
        int64_t i = rows ? rows[r] : r;
        double acc = 0.0;
        for (int64_t j = 0; j < nt; ++j)
            acc += laplace_entry(&m, i, j) * x[j];
        y[r] = acc / (4.0 * OR_PI);
    }
    mesh_free(&m);
    return 0;
}

/* y = A t for the Stokes single layer, u_i = -1/(8 pi mu) sum_j int_j G t_j,
 * vectors as [nt][3]. */
int or_matvec_stokes(int64_t nt, const double *xyz, const int32_t *tri, double mu,
                     const double *x, double *y, int64_t nrows, const int64_t *rows)
{
    mesh_t m;
    if (mesh_init(&m, nt, xyz, tri))
        return -1;
    int64_t nr = rows ? nrows : nt;
    double pref = -1.0 / (8.0 * OR_PI * mu);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nr; ++r) {
        int64_t i = rows ? rows[r] : r;
        double acc[3] = {0, 0, 0}, G[9];
        for (int64_t j = 0; j < nt; ++j) {
            stokes_entry(&m, i, j, G);
            for (int p = 0; p < 3; ++p)
                acc[p] += (G[3 * p] * x[3 * j] + G[3 * p + 1] * x[3 * j + 1]) + G[3 * p + 2] * x[3 * j + 2];
        }
        for (int p = 0; p < 3; ++p)
            y[3 * r + p] = pref * acc[p];
    }
    mesh_free(&m);
    return 0;
}

/* y = (1/2 I - K) x, the second-kind operator of the exterior Neumann problem:
 * y_i = x_i / 2 - (1/4pi) sum_j x_j int_j n_j . (x_i - y) / |x_i - y|^3. */
int or_matvec_laplace_dl(int64_t nt, const double *xyz, const int32_t *tri,
                         const double *x, double *y, int64_t nrows, const int64_t *rows)
{
    mesh_t m;
    if (mesh_init(&m, nt, xyz, tri))
        return -1;
    int64_t nr = rows ? nrows : nt;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nr; ++r) {
        int64_t i = rows ? rows[r] : r;
        double acc = 0.0;
        for (int64_t j = 0; j < nt; ++j)
            acc += dl_entry(&m, i, j) * x[j];
        y[r] = 0.5 * x[i] - acc / (4.0 * OR_PI);
    }
    mesh_free(&m);
    return 0;
}

double or_laplace_dl_entry(int64_t nt, const double *xyz, const int32_t *tri, int64_t i, int64_t j)
{
    mesh_t m;
    if (mesh_init(&m, nt, xyz, tri))
        return NAN;
    double v = dl_entry(&m, i, j);
    mesh_free(&m);
    return v;
}

/* Single entries, for tests: the Laplace entry int_j 1/r and the Stokes block. */
double or_laplace_entry(int64_t nt, const double *xyz, const int32_t *tri, int64_t i, int64_t j)
{
    mesh_t m;
    if (mesh_init(&m, nt, xyz, tri))
        return NAN;
    double v = laplace_entry(&m, i, j);
    mesh_free(&m);
    return v;
}

/* Row i of the Laplace operator before the 1/(4 pi) factor: out[j] = int_j 1/r, and
 * the class of each entry (0 far, 1 near-singular, 2 self). */
int or_laplace_row(int64_t nt, const double *xyz, const int32_t *tri, int64_t i, double *out,
                   int32_t *cls)
{
    mesh_t m;
    if (mesh_init(&m, nt, xyz, tri))
        return -1;
    for (int64_t j = 0; j < nt; ++j) {
        out[j] = laplace_entry(&m, i, j);
        if (cls)
            cls[j] = classify(&m, i, j);
    }
    mesh_free(&m);
    return 0;
}

int or_classify(int64_t nt, const double *xyz, const int32_t *tri, int64_t i, int64_t j)
{
    mesh_t m;
    if (mesh_init(&m, nt, xyz, tri))
        return -1;
    int c = classify(&m, i, j);
    mesh_free(&m);
    return c;
}

/* ------------------------------------------------------------------------- */
/* GMRES(m) (Sec. 2.4), unpreconditioned, modified Gram-Schmidt, Givens.      */
/* x0 = 0.  The stopping test uses the implicit relative residual            */
/* |g_{k+1}| / |b|; at a restart and at the end the true residual b - A x is  */
/* formed.  Returns 0 when converged, 1 when max_iter was reached.            */
/* ------------------------------------------------------------------------- */
typedef void (*or_mv_fn)(void *user, const double *x, double *y);

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += a[i] * b[i];
    return s;
}

int or_gmres(int64_t n, or_mv_fn mv, void *user, const double *b, double tol,
             int restart, int max_iter, double *x, double *res_hist, int hist_cap,
             int *iters_out, double *true_res_out)
{
    int m = restart;
    double *V = (double *)calloc((size_t)(m + 1) * (size_t)n, sizeof(double));
    double *H = (double *)calloc((size_t)(m + 1) * (size_t)m, sizeof(double));
    double *cs = (double *)calloc((size_t)m, sizeof(double));
    double *sn = (double *)calloc((size_t)m, sizeof(double));
    double *g = (double *)calloc((size_t)m + 1, sizeof(double));
    double *r = (double *)calloc((size_t)n, sizeof(double));
    double *w = (double *)calloc((size_t)n, sizeof(double));
    double *yv = (double *)calloc((size_t)m, sizeof(double));
    if (!V || !H || !cs || !sn || !g || !r || !w || !yv)
        return -1;
    for (int64_t i = 0; i < n; ++i)
        x[i] = 0.0;
    double bnorm = sqrt(dot(n, b, b));
    int it = 0, converged = 0;
    double rel = 1.0;
    if (bnorm == 0.0) {
        converged = 1;
        rel = 0.0;
    }
    memcpy(r, b, sizeof(double) * (size_t)n);
    while (!converged && it < max_iter) {
        double beta = sqrt(dot(n, r, r));
        if (beta / bnorm <= tol) {
            converged = 1;
            break;
        }
        for (int64_t i = 0; i < n; ++i)
            V[i] = r[i] / beta;
        for (int k = 0; k <= m; ++k)
            g[k] = 0.0;
        g[0] = beta;
        int k;
        for (k = 0; k < m && it < max_iter; ++k) {
            double *vk = V + (size_t)k * n, *vn = V + (size_t)(k + 1) * n;
            mv(user, vk, w);
            for (int j = 0; j <= k; ++j) {
                double *vj = V + (size_t)j * n;
                double h = dot(n, w, vj);
                H[(size_t)j * m + k] = h;
                for (int64_t i = 0; i < n; ++i)
                    w[i] -= h * vj[i];
            }
            double hn = sqrt(dot(n, w, w));
            H[(size_t)(k + 1) * m + k] = hn;
            if (hn != 0.0)
                for (int64_t i = 0; i < n; ++i)
                    vn[i] = w[i] / hn;
            /* apply previous rotations to column k */
            for (int j = 0; j < k; ++j) {
                double a = H[(size_t)j * m + k], c2 = H[(size_t)(j + 1) * m + k];
                H[(size_t)j * m + k] = cs[j] * a + sn[j] * c2;
                H[(size_t)(j + 1) * m + k] = -sn[j] * a + cs[j] * c2;
            }
            double a = H[(size_t)k * m + k], c2 = H[(size_t)(k + 1) * m + k];
            double den = sqrt(a * a + c2 * c2);
            cs[k] = den == 0.0 ? 1.0 : a / den;
            sn[k] = den == 0.0 ? 0.0 : c2 / den;
            H[(size_t)k * m + k] = den;
            H[(size_t)(k + 1) * m + k] = 0.0;
            g[k + 1] = -sn[k] * g[k];
            g[k] = cs[k] * g[k];
            rel = fabs(g[k + 1]) / bnorm;
            if (res_hist && it < hist_cap)
                res_hist[it] = rel;
            ++it;
            if (rel <= tol || hn == 0.0) {
                ++k;
                break;
            }
        }
        /* back substitution H y = g, x += V y */
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int j = i + 1; j < k; ++j)
                s -= H[(size_t)i * m + j] * yv[j];
            yv[i] = s / H[(size_t)i * m + i];
        }
        for (int j = 0; j < k; ++j) {
            double *vj = V + (size_t)j * n;
            for (int64_t i = 0; i < n; ++i)
                x[i] += yv[j] * vj[i];
        }
        /* true residual */
        mv(user, x, w);
        for (int64_t i = 0; i < n; ++i)
            r[i] = b[i] - w[i];
        double tr = sqrt(dot(n, r, r)) / bnorm;
        if (rel <= tol || tr <= tol)
            converged = 1;
    }
    if (true_res_out) {
        mv(user, x, w);
        for (int64_t i = 0; i < n; ++i)
            r[i] = b[i] - w[i];
        *true_res_out = bnorm == 0.0 ? 0.0 : sqrt(dot(n, r, r)) / bnorm;
    }
    if (iters_out)
        *iters_out = it;
    free(V); free(H); free(cs); free(sn); free(g); free(r); free(w); free(yv);
    return converged ? 0 : 1;
}

/* Dense-operator GMRES solves on a mesh. */
typedef struct {
    int64_t nt;
    const double *xyz;
    const int32_t *tri;
    double mu;
} solve_ctx;

static void mv_laplace(void *u, const double *x, double *y)
{
    solve_ctx *s = (solve_ctx *)u;
    or_matvec_laplace(s->nt, s->xyz, s->tri, x, y, 0, NULL);
}

static void mv_stokes(void *u, const double *x, double *y)
{
    solve_ctx *s = (solve_ctx *)u;
    or_matvec_stokes(s->nt, s->xyz, s->tri, s->mu, x, y, 0, NULL);
}

static void mv_laplace_dl(void *u, const double *x, double *y)
{
    solve_ctx *s = (solve_ctx *)u;
    or_matvec_laplace_dl(s->nt, s->xyz, s->tri, x, y, 0, NULL);
}

int or_solve(int kernel, int64_t nt, const double *xyz, const int32_t *tri, double mu,
             const double *b, double tol, int restart, int max_iter, double *x,
             double *res_hist, int hist_cap, int *iters, double *true_res)
{
    solve_ctx s = {nt, xyz, tri, mu};
    int64_t n = kernel == 1 ? 3 * nt : nt;
    or_mv_fn mv = kernel == 0 ? mv_laplace : kernel == 1 ? mv_stokes : mv_laplace_dl;
    return or_gmres(n, mv, &s, b, tol, restart, max_iter, x, res_hist, hist_cap, iters, true_res);
}

/* Drag and torque (Eq. 20): F = sum_j t_j S_j, T = sum_j c_j x t_j S_j. */
void or_force_torque(int64_t nt, const double *xyz, const int32_t *tri, const double *t,
                     double *F, double *T)
{
    double c[3], S;
    for (int d = 0; d < 3; ++d)
        F[d] = T[d] = 0.0;
    for (int64_t j = 0; j < nt; ++j) {
        const int32_t *tr = tri + 3 * j;
        panel_geom(xyz + 3 * (int64_t)tr[0], xyz + 3 * (int64_t)tr[1], xyz + 3 * (int64_t)tr[2], c, &S, NULL);
        const double *tj = t + 3 * j;
        for (int d = 0; d < 3; ++d)
            F[d] += tj[d] * S;
        T[0] += (c[1] * tj[2] - c[2] * tj[1]) * S;
        T[1] += (c[2] * tj[0] - c[0] * tj[2]) * S;
        T[2] += (c[0] * tj[1] - c[1] * tj[0]) * S;
    }
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

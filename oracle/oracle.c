/*
 * FP64 CPU ORACLE for the node-patch boundary-integral Poisson-Boltzmann
 * operator (Zhang, DeBuhr, Niedzielski, Mayolo, Lu, Sterling, "DASHMM
 * accelerated adaptive fast multipole Poisson-Boltzmann solver on distributed
 * memory architecture", Section 2).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header or table with the GPU path.
 *
 * What it computes, plainly and slowly, in double precision:
 *   - patch geometry of the node-patch scheme (Section 2, Figure 1);
 *   - the kernels G, u and their normal derivatives (Section 2, Eq. 3);
 *   - the near set and the patch integrals A, B, C, D of Eq. (6);
 *   - the direct O(N^2) matrix-vector product of the block system Eq. (5),
 *     point rule for far pairs, patch integrals for near pairs;
 *   - the right-hand side of Eq. (5) and the reaction-field energy.
 * GMRES, the tree and the closed forms live in the Python half (oracle.py).
 *
 * Built with -O2 -ffp-contract=off so that no multiply-add is fused.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define FOUR_PI 12.566370614359172953850573533118

/* ------------------------------------------------------------------------ */
/* Kernels (Section 2, Eq. 3).  R = x - y, x the target (node p, normal nx),  */
/* y the source (on patch t, normal ny).                                      */
/* ------------------------------------------------------------------------ */

/* a(s) = 1 - e^{-s}(1+s), b(s) = 3 - e^{-s}(3+3s+s^2): the factors that remain
 * of the second normal derivative when the screened kernel is subtracted from
 * the Laplace one.  Power series below s = 0.1 (no cancellation), long double
 * closed form above. */
static double fac_a(double s)
{
    if (s < 0.1) {
        /* a(s) = sum_{k>=2} (-1)^k (k-1) s^k / k! */
        long double sum = 0.0L, term = 1.0L;
        for (int k = 1; k <= 12; ++k) {
            term *= (long double)s / k;            /* s^k / k! */
            if (k >= 2) sum += ((k & 1) ? -1.0L : 1.0L) * (k - 1) * term;
        }
        return (double)sum;
    }
    long double e = expl(-(long double)s);
    return (double)(1.0L - e * (1.0L + s));
}

static double fac_b(double s)
{
    if (s < 0.1) {
        /* b(s) = -sum_{k>=1} (-1)^k (k-1)(k-3) s^k / k! */
        long double sum = 0.0L, term = 1.0L;
        for (int k = 1; k <= 12; ++k) {
            term *= (long double)s / k;
            sum -= ((k & 1) ? -1.0L : 1.0L) * (long double)((k - 1) * (k - 3)) * term;
        }
        return (double)sum;
    }
    long double e = expl(-(long double)s);
    long double ls = s;
    return (double)(3.0L - e * (3.0L + 3.0L * ls + ls * ls));
}

/* out[0..9] = G, u, dG/dny, du/dny, dG/dnx, du/dnx, d2G/dnx dny, d2u/dnx dny,
 *             G-u (cancellation-free), d2G-d2u (cancellation-free). */
void orc_kernels(const double *x, const double *nx, const double *y,
                 const double *ny, double kappa, double *out)
{
    double R[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
    double r2 = (R[0] * R[0] + R[1] * R[1]) + R[2] * R[2];
    double r = sqrt(r2);
    double kr = kappa * r;
    double e = exp(-kr);
    double Rny = (R[0] * ny[0] + R[1] * ny[1]) + R[2] * ny[2];
    double Rnx = (R[0] * nx[0] + R[1] * nx[1]) + R[2] * nx[2];
    double nxny = (nx[0] * ny[0] + nx[1] * ny[1]) + nx[2] * ny[2];
    double r3 = r2 * r, r5 = r3 * r2;
    out[0] = 1.0 / (FOUR_PI * r);
    out[1] = e / (FOUR_PI * r);
    out[2] = Rny / (FOUR_PI * r3);
    out[3] = e * (1.0 + kr) * Rny / (FOUR_PI * r3);
    out[4] = -Rnx / (FOUR_PI * r3);
    out[5] = -e * (1.0 + kr) * Rnx / (FOUR_PI * r3);
    out[6] = (nxny / r3 - 3.0 * Rnx * Rny / r5) / FOUR_PI;
    out[7] = e * ((1.0 + kr) * nxny / r3 - (3.0 + 3.0 * kr + kr * kr) * Rnx * Rny / r5) / FOUR_PI;
    out[8] = -expm1(-kr) / (FOUR_PI * r);
    out[9] = (nxny * fac_a(kr) / r3 - Rnx * Rny * fac_b(kr) / r5) / FOUR_PI;
}

/* The four integrands of Eq. (6) at one source point y (normal ny) for target
 * x (normal nx): acc[0..3] += w * {A, B, C, D} integrand. */
static void abcd_integrand(const double *x, const double *nx, const double *y,
                           const double *ny, double kappa, double inv_ebar,
                           double w, double *acc)
{
    double k[10];
    orc_kernels(x, nx, y, ny, kappa, k);
    acc[0] += w * k[8];                               /* G - u               */
    acc[1] += w * (inv_ebar * k[2] - k[3]);           /* dG/dn/eb - du/dn    */
    acc[2] += w * (k[4] - inv_ebar * k[5]);           /* dG/dn0 - du/dn0/eb  */
    acc[3] += w * (inv_ebar * k[9]);                  /* (d2G - d2u)/eb      */
}

/* ------------------------------------------------------------------------ */
/* Geometry of the node-patch scheme (Section 2, Figure 1)                   */
/* ------------------------------------------------------------------------ */

static double dist2(const double *a, const double *b)
{
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return (dx * dx + dy * dy) + dz * dz;
}

/* Triangle areas and unit normals; node patch areas (one third of each
 * incident triangle: the dual cell bounded by edge midpoints and centroids);
 * node normals (area-weighted facet normals, normalised); squared patch radius
 * (largest squared distance from the node to the patch's midpoints/centroids). */
void orc_geometry(long n, const double *V, long m, const int *T,
                  double *tri_area, double *tri_n, double *node_area,
                  double *node_n, double *rho2)
{
    memset(node_area, 0, sizeof(double) * n);
    memset(node_n, 0, sizeof(double) * 3 * n);
    memset(rho2, 0, sizeof(double) * n);
    for (long k = 0; k < m; ++k) {
        const double *a = V + 3 * (long)T[3 * k], *b = V + 3 * (long)T[3 * k + 1],
                     *c = V + 3 * (long)T[3 * k + 2];
        double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                        e1[0] * e2[1] - e1[1] * e2[0]};
        double len = sqrt((cr[0] * cr[0] + cr[1] * cr[1]) + cr[2] * cr[2]);
        double A = 0.5 * len;
        tri_area[k] = A;
        for (int d = 0; d < 3; ++d) tri_n[3 * k + d] = cr[d] / len;
        double cen[3];
        for (int d = 0; d < 3; ++d) cen[d] = ((a[d] + b[d]) + c[d]) / 3.0;
        for (int j = 0; j < 3; ++j) {
            long v = T[3 * k + j];
            node_area[v] += A / 3.0;
            for (int d = 0; d < 3; ++d) node_n[3 * v + d] += A * tri_n[3 * k + d];
            const double *pv = V + 3 * v;
            /* the two edges of this triangle incident to v */
            for (int jj = 1; jj <= 2; ++jj) {
                const double *pu = V + 3 * (long)T[3 * k + (j + jj) % 3];
                double mid[3] = {(pv[0] + pu[0]) * 0.5, (pv[1] + pu[1]) * 0.5,
                                 (pv[2] + pu[2]) * 0.5};
                double d2 = dist2(mid, pv);
                if (d2 > rho2[v]) rho2[v] = d2;
            }
            double d2 = dist2(cen, pv);
            if (d2 > rho2[v]) rho2[v] = d2;
        }
    }
    for (long v = 0; v < n; ++v) {
        double *q = node_n + 3 * v;
        double l = sqrt((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]);
        q[0] /= l; q[1] /= l; q[2] /= l;
    }
}

/* ------------------------------------------------------------------------ */
/* Near set (tree-independent distance rule)                                 */
/* N(p) = {p} U {t : |x_p - x_t|^2 < eta^2 max(rho_p^2, rho_t^2)}           */
/* ------------------------------------------------------------------------ */

static int is_near(const double *V, const double *rho2, double eta2, long p, long t)
{
    if (p == t) return 1;
    double d2 = dist2(V + 3 * p, V + 3 * t);
    double r2 = rho2[p] > rho2[t] ? rho2[p] : rho2[t];
    return d2 < eta2 * r2;
}

/* Count near columns of each requested row (brute force over all nodes). */
void orc_near_count(long n, const double *V, const double *rho2, double eta,
                    long nrows, const long *rows, long *count)
{
    double eta2 = eta * eta;
#pragma omp parallel for schedule(dynamic, 16)
    for (long i = 0; i < nrows; ++i) {
        long c = 0;
        for (long t = 0; t < n; ++t) c += is_near(V, rho2, eta2, rows[i], t);
        count[i] = c;
    }
}

/* Fill near columns (ascending) of each requested row; ptr has nrows+1. */
void orc_near_fill(long n, const double *V, const double *rho2, double eta,
                   long nrows, const long *rows, const long *ptr, long *col)
{
    double eta2 = eta * eta;
#pragma omp parallel for schedule(dynamic, 16)
    for (long i = 0; i < nrows; ++i) {
        long c = ptr[i];
        for (long t = 0; t < n; ++t)
            if (is_near(V, rho2, eta2, rows[i], t)) col[c++] = t;
    }
}

/* ------------------------------------------------------------------------ */
/* Patch integrals of Eq. (6) over Delta S_t                                 */
/* ------------------------------------------------------------------------ */

#define NQ_NEAR 8      /* Gauss points per direction on a leaf sub-triangle */
#define NQ_SELF 16     /* Gauss points per direction for the singular patch */
#define REFINE 2.0     /* split while |x_p - centroid| < REFINE * diameter  */
#define MAX_DEPTH 10

static double gl_x[32][32], gl_w[32][32];
static int gl_ready[32];

/* Gauss-Legendre nodes/weights on [0,1] by Newton iteration on P_n. */
static void gauss_legendre(int nq)
{
    if (gl_ready[nq]) return;
    for (int i = 0; i < nq; ++i) {
        double z = cos(M_PI * (i + 0.75) / (nq + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= nq; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            dp = nq * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= nq; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            dp = nq * (z * p1 - p0) / (z * z - 1.0);
        }
        gl_x[nq][i] = 0.5 * (1.0 - z);
        gl_w[nq][i] = 1.0 / ((1.0 - z * z) * dp * dp);   /* = 2/((1-z^2)P'^2) / 2 */
    }
    gl_ready[nq] = 1;
}

/* Collapsed Gauss product rule on triangle (P0,P1,P2) with the collapse at P0:
 * y = P0 + u (P1-P0) + u v (P2-P1), dS = 2|tau| u du dv. */
static void tri_rule(const double *x, const double *nx, const double *P0,
                     const double *P1, const double *P2, const double *ny,
                     double area, double kappa, double inv_ebar, int nq,
                     int self, double *acc)
{
    for (int i = 0; i < nq; ++i) {
        double u = gl_x[nq][i];
        for (int j = 0; j < nq; ++j) {
            double v = gl_x[nq][j];
            double w = 2.0 * area * u * gl_w[nq][i] * gl_w[nq][j];
            double y[3];
            for (int d = 0; d < 3; ++d)
                y[d] = P0[d] + u * (P1[d] - P0[d]) + u * v * (P2[d] - P1[d]);
            if (self) {
                /* Flat-facet reading on the node's own patch: the target
                 * normal is the facet normal, so R.n = 0 and only the G-u and
                 * second-derivative terms survive. */
                double k[10];
                orc_kernels(x, ny, y, ny, kappa, k);
                acc[0] += w * k[8];
                acc[3] += w * inv_ebar * k[9];
            } else {
                abcd_integrand(x, nx, y, ny, kappa, inv_ebar, w, acc);
            }
        }
    }
}

static double tri_area3(const double *a, const double *b, const double *c)
{
    double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                    e1[0] * e2[1] - e1[1] * e2[0]};
    return 0.5 * sqrt((cr[0] * cr[0] + cr[1] * cr[1]) + cr[2] * cr[2]);
}

/* Adaptive midpoint subdivision: a sub-triangle is split into its four
 * midpoint children while the target is closer than REFINE diameters to its
 * centroid; leaves get the NQ_NEAR x NQ_NEAR collapsed Gauss rule. */
static void adapt(const double *x, const double *nx, const double *P0,
                  const double *P1, const double *P2, const double *ny,
                  double kappa, double inv_ebar, int depth, double *acc)
{
    double c[3], diam2;
    for (int d = 0; d < 3; ++d) c[d] = ((P0[d] + P1[d]) + P2[d]) / 3.0;
    diam2 = dist2(P0, P1);
    if (dist2(P1, P2) > diam2) diam2 = dist2(P1, P2);
    if (dist2(P2, P0) > diam2) diam2 = dist2(P2, P0);
    if (depth < MAX_DEPTH && dist2(x, c) < REFINE * REFINE * diam2) {
        double m01[3], m12[3], m20[3];
        for (int d = 0; d < 3; ++d) {
            m01[d] = (P0[d] + P1[d]) * 0.5;
            m12[d] = (P1[d] + P2[d]) * 0.5;
            m20[d] = (P2[d] + P0[d]) * 0.5;
        }
        adapt(x, nx, P0, m01, m20, ny, kappa, inv_ebar, depth + 1, acc);
        adapt(x, nx, m01, P1, m12, ny, kappa, inv_ebar, depth + 1, acc);
        adapt(x, nx, m20, m12, P2, ny, kappa, inv_ebar, depth + 1, acc);
        adapt(x, nx, m12, m20, m01, ny, kappa, inv_ebar, depth + 1, acc);
        return;
    }
    tri_rule(x, nx, P0, P1, P2, ny, tri_area3(P0, P1, P2), kappa, inv_ebar,
             NQ_NEAR, 0, acc);
}

/* {A,B,C,D}_{pt} of Eq. (6) as integrals over the patch of node t.  The patch
 * is the union, over triangles T = (t,u,w) incident to t, of the flat pieces
 * (t, m_tu, c_T) and (t, c_T, m_tw) that carry the facet normal of T. */
void orc_patch_coeffs(long n, const double *V, long m, const int *T,
                      const double *tri_n, const double *node_n,
                      const long *inc_ptr, const long *inc_tri,
                      double kappa, double ebar, long npairs, const long *pp,
                      const long *tt, double *out /* npairs x 4 */)
{
    (void)n; (void)m;
    gauss_legendre(NQ_NEAR);
    gauss_legendre(NQ_SELF);
    double inv_ebar = 1.0 / ebar;
#pragma omp parallel for schedule(dynamic, 8)
    for (long q = 0; q < npairs; ++q) {
        long p = pp[q], t = tt[q];
        const double *x = V + 3 * p, *nx = node_n + 3 * p, *vt = V + 3 * t;
        double acc[4] = {0, 0, 0, 0};
        for (long k = inc_ptr[t]; k < inc_ptr[t + 1]; ++k) {
            long tri = inc_tri[k];
            const int *tv = T + 3 * tri;
            int j = (tv[0] == t) ? 0 : (tv[1] == t) ? 1 : 2;
            const double *pu = V + 3 * (long)tv[(j + 1) % 3];
            const double *pw = V + 3 * (long)tv[(j + 2) % 3];
            const double *a = V + 3 * (long)tv[0], *b = V + 3 * (long)tv[1],
                         *c = V + 3 * (long)tv[2];
            double cen[3], mu[3], mw[3];
            for (int d = 0; d < 3; ++d) {
                cen[d] = ((a[d] + b[d]) + c[d]) / 3.0;
                mu[d] = (vt[d] + pu[d]) * 0.5;
                mw[d] = (vt[d] + pw[d]) * 0.5;
            }
            const double *ny = tri_n + 3 * tri;
            if (p == t) {
                tri_rule(x, nx, vt, mu, cen, ny, tri_area3(vt, mu, cen), kappa,
                         inv_ebar, NQ_SELF, 1, acc);
                tri_rule(x, nx, vt, cen, mw, ny, tri_area3(vt, cen, mw), kappa,
                         inv_ebar, NQ_SELF, 1, acc);
            } else {
                adapt(x, nx, vt, mu, cen, ny, kappa, inv_ebar, 0, acc);
                adapt(x, nx, vt, cen, mw, ny, kappa, inv_ebar, 0, acc);
            }
        }
        for (int d = 0; d < 4; ++d) out[4 * q + d] = acc[d];
    }
}

/* Point-rule coefficients for a far pair (integrand constant on the patch,
 * taken at node t with the node normal, times the patch area). */
static void point_coeffs(const double *V, const double *node_n,
                         const double *node_area, double kappa, double inv_ebar,
                         long p, long t, double *c4)
{
    c4[0] = c4[1] = c4[2] = c4[3] = 0.0;
    abcd_integrand(V + 3 * p, node_n + 3 * p, V + 3 * t, node_n + 3 * t, kappa,
                   inv_ebar, node_area[t], c4);
}

void orc_point_coeffs(const double *V, const double *node_n,
                      const double *node_area, double kappa, double ebar,
                      long npairs, const long *pp, const long *tt, double *out)
{
    for (long q = 0; q < npairs; ++q)
        point_coeffs(V, node_n, node_area, kappa, 1.0 / ebar, pp[q], tt[q],
                     out + 4 * q);
}

/* ------------------------------------------------------------------------ */
/* Direct matrix-vector product of Eq. (5)                                   */
/*   y_f(p) = alpha f_p + sum_t B_pt f_t - sum_t A_pt h_t                    */
/*   y_h(p) = alpha h_p + sum_t D_pt f_t - sum_t C_pt h_t                    */
/* alpha = 1/(2 ebar) + 1/2.  Near columns (sorted CSR per requested row)    */
/* take the stored patch integrals; all other columns the point rule.        */
/* x = [f(0..n-1); h(0..n-1)];  y has 2 values per requested row (yf, yh).   */
/* ------------------------------------------------------------------------ */
void orc_matvec_rows(long n, const double *V, const double *node_n,
                     const double *node_area, double kappa, double ebar,
                     long nrows, const long *rows, const long *near_ptr,
                     const long *near_col, const double *near_coef,
                     const double *x, double *y)
{
    double inv_ebar = 1.0 / ebar;
    double alpha = 0.5 / ebar + 0.5;
    const double *f = x, *h = x + n;
#pragma omp parallel for schedule(dynamic, 4)
    for (long i = 0; i < nrows; ++i) {
        long p = rows[i];
        long k = near_ptr[i], kend = near_ptr[i + 1];
        double yf = 0.0, yh = 0.0;
        for (long t = 0; t < n; ++t) {
            double c4[4];
            if (k < kend && near_col[k] == t) {
                c4[0] = near_coef[4 * k]; c4[1] = near_coef[4 * k + 1];
                c4[2] = near_coef[4 * k + 2]; c4[3] = near_coef[4 * k + 3];
                ++k;
            } else {
                point_coeffs(V, node_n, node_area, kappa, inv_ebar, p, t, c4);
            }
            yf += c4[1] * f[t] - c4[0] * h[t];
            yh += c4[3] * f[t] - c4[2] * h[t];
        }
        y[2 * i] = alpha * f[p] + yf;
        y[2 * i + 1] = alpha * h[p] + yh;
    }
}

/* ------------------------------------------------------------------------ */
/* Right-hand side of Eq. (5): b_f = (1/eps_s) sum_k q_k G(p,k),             */
/* b_h = (1/eps_s) sum_k q_k dG(p,k)/dn_p (derivative at the node, along n_p)*/
/* ------------------------------------------------------------------------ */
void orc_rhs(long n, const double *V, const double *node_n, long na,
             const double *ax, const double *q, double eps_s, double *b)
{
#pragma omp parallel for schedule(static)
    for (long p = 0; p < n; ++p) {
        double sf = 0.0, sh = 0.0;
        for (long k = 0; k < na; ++k) {
            double R[3] = {V[3 * p] - ax[3 * k], V[3 * p + 1] - ax[3 * k + 1],
                           V[3 * p + 2] - ax[3 * k + 2]};
            double r2 = (R[0] * R[0] + R[1] * R[1]) + R[2] * R[2];
            double r = sqrt(r2);
            double Rn = (R[0] * node_n[3 * p] + R[1] * node_n[3 * p + 1]) +
                        R[2] * node_n[3 * p + 2];
            sf += q[k] / (FOUR_PI * r);
            sh += -q[k] * Rn / (FOUR_PI * r2 * r);
        }
        b[p] = sf / eps_s;
        b[n + p] = sh / eps_s;
    }
}

/* ------------------------------------------------------------------------ */
/* Reaction potential at the atoms from the interior Green representation,   */
/* point rule on each patch:                                                 */
/*   phi_reac(r_k) = sum_t a_t [ebar h_t G(r_k,r_t) - f_t dG(r_k,r_t)/dn_t]  */
/* Returns sum_k q_k phi_reac(r_k) (internal units).                         */
/* ------------------------------------------------------------------------ */
double orc_energy_sum(long n, const double *V, const double *node_n,
                      const double *node_area, long na, const double *ax,
                      const double *q, double ebar, const double *f,
                      const double *h, double *phi /* na, may be NULL */)
{
    double total = 0.0;
    double *tmp = (double *)malloc(sizeof(double) * (na > 0 ? na : 1));
#pragma omp parallel for schedule(static)
    for (long k = 0; k < na; ++k) {
        double s = 0.0;
        for (long t = 0; t < n; ++t) {
            double R[3] = {ax[3 * k] - V[3 * t], ax[3 * k + 1] - V[3 * t + 1],
                           ax[3 * k + 2] - V[3 * t + 2]};
            double r2 = (R[0] * R[0] + R[1] * R[1]) + R[2] * R[2];
            double r = sqrt(r2);
            double Rn = (R[0] * node_n[3 * t] + R[1] * node_n[3 * t + 1]) +
                        R[2] * node_n[3 * t + 2];
            double G = 1.0 / (FOUR_PI * r);
            double dGdn = Rn / (FOUR_PI * r2 * r);
            s += node_area[t] * (ebar * h[t] * G - f[t] * dGdn);
        }
        tmp[k] = s;
    }
    for (long k = 0; k < na; ++k) {
        if (phi) phi[k] = tmp[k];
        total += q[k] * tmp[k];
    }
    free(tmp);
    return total;
}

/* ------------------------------------------------------------------------ */
/* Thread count of the parallel loops above (for timing the oracle)          */
/* ------------------------------------------------------------------------ */

void orc_set_threads(int n) { omp_set_num_threads(n); }

int orc_max_threads(void) { return omp_get_max_threads(); }

/* Host-side driver for the oracle's C library under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built by tests/test_oracle_sanitized.py with
 * gcc, never for a GPU).  It reads a small problem from a binary file, runs
 * every oracle entry point on it (geometry, near set, patch and point
 * coefficients, direct matvec rows, right-hand side, energy sum) and writes
 * the results, which the test compares with the unsanitized library's.
 *
 * Input (native endianness): int64 n, m, na; double kappa, ebar, eps_s, eta;
 * double V[3n]; int32 T[3m]; int64 inc_ptr[n+1]; int64 inc_tri[3m];
 * double ax[3na], q[na], x[2n].
 * Output: double tri_area[m], tri_n[3m], area[n], normal[3n], rho2[n];
 * int64 nnz, ptr[n+1], col[nnz]; double coef[4 nnz], point[4 nnz], y[2n],
 * b[2n], esum, phi[na]. */
#include <stdio.h>
#include <stdlib.h>

void orc_geometry(long n, const double *V, long m, const int *T, double *tri_area,
                  double *tri_n, double *node_area, double *node_n, double *rho2);
void orc_near_count(long n, const double *V, const double *rho2, double eta, long nrows,
                    const long *rows, long *count);
void orc_near_fill(long n, const double *V, const double *rho2, double eta, long nrows,
                   const long *rows, const long *ptr, long *col);
void orc_patch_coeffs(long n, const double *V, long m, const int *T, const double *tri_n,
                      const double *node_n, const long *inc_ptr, const long *inc_tri,
                      double kappa, double ebar, long npairs, const long *pp, const long *tt,
                      double *out);
void orc_point_coeffs(const double *V, const double *node_n, const double *node_area,
                      double kappa, double ebar, long npairs, const long *pp, const long *tt,
                      double *out);
void orc_matvec_rows(long n, const double *V, const double *node_n, const double *node_area,
                     double kappa, double ebar, long nrows, const long *rows,
                     const long *near_ptr, const long *near_col, const double *near_coef,
                     const double *x, double *y);
void orc_rhs(long n, const double *V, const double *node_n, long na, const double *ax,
             const double *q, double eps_s, double *b);
double orc_energy_sum(long n, const double *V, const double *node_n, const double *node_area,
                      long na, const double *ax, const double *q, double ebar, const double *f,
                      const double *h, double *phi);

static void *take(FILE *f, size_t count, size_t size) {
    void *p = malloc(count * size + 1);
    if (!p || fread(p, size, count, f) != count) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
    return p;
}

static void put(FILE *f, const void *p, size_t count, size_t size) {
    if (fwrite(p, size, count, f) != count) {
        fprintf(stderr, "short output\n");
        exit(2);
    }
}

int main(int argc, char **argv) {
    if (argc != 3) {
        fprintf(stderr, "usage: %s input output\n", argv[0]);
        return 2;
    }
    FILE *in = fopen(argv[1], "rb");
    if (!in) return 2;
    long long *hdr = take(in, 3, sizeof(long long));
    const long n = (long)hdr[0], m = (long)hdr[1], na = (long)hdr[2];
    double *par = take(in, 4, sizeof(double));
    const double kappa = par[0], ebar = par[1], eps_s = par[2], eta = par[3];
    double *V = take(in, 3 * n, sizeof(double));
    int *T = take(in, 3 * m, sizeof(int));
    long *inc_ptr = take(in, n + 1, sizeof(long));
    long *inc_tri = take(in, 3 * m, sizeof(long));
    double *ax = take(in, 3 * na, sizeof(double));
    double *q = take(in, na, sizeof(double));
    double *x = take(in, 2 * n, sizeof(double));
    fclose(in);

    double *ta = malloc(sizeof(double) * m), *tn = malloc(sizeof(double) * 3 * m);
    double *area = malloc(sizeof(double) * n), *nn = malloc(sizeof(double) * 3 * n);
    double *rho2 = malloc(sizeof(double) * n);
    orc_geometry(n, V, m, T, ta, tn, area, nn, rho2);

    long *rows = malloc(sizeof(long) * n), *cnt = malloc(sizeof(long) * n);
    long *ptr = malloc(sizeof(long) * (n + 1));
    for (long i = 0; i < n; ++i) rows[i] = i;
    orc_near_count(n, V, rho2, eta, n, rows, cnt);
    ptr[0] = 0;
    for (long i = 0; i < n; ++i) ptr[i + 1] = ptr[i] + cnt[i];
    const long nnz = ptr[n];
    long *col = malloc(sizeof(long) * nnz), *pp = malloc(sizeof(long) * nnz);
    orc_near_fill(n, V, rho2, eta, n, rows, ptr, col);
    for (long i = 0; i < n; ++i)
        for (long k = ptr[i]; k < ptr[i + 1]; ++k) pp[k] = i;

    double *coef = malloc(sizeof(double) * 4 * nnz), *point = malloc(sizeof(double) * 4 * nnz);
    orc_patch_coeffs(n, V, m, T, tn, nn, inc_ptr, inc_tri, kappa, ebar, nnz, pp, col, coef);
    orc_point_coeffs(V, nn, area, kappa, ebar, nnz, pp, col, point);

    double *y = malloc(sizeof(double) * 2 * n), *b = malloc(sizeof(double) * 2 * n);
    double *phi = malloc(sizeof(double) * (na + 1));
    orc_matvec_rows(n, V, nn, area, kappa, ebar, n, rows, ptr, col, coef, x, y);
    orc_rhs(n, V, nn, na, ax, q, eps_s, b);
    const double esum = orc_energy_sum(n, V, nn, area, na, ax, q, ebar, x, x + n, phi);

    FILE *out = fopen(argv[2], "wb");
    if (!out) return 2;
    put(out, ta, m, sizeof(double));
    put(out, tn, 3 * m, sizeof(double));
    put(out, area, n, sizeof(double));
    put(out, nn, 3 * n, sizeof(double));
    put(out, rho2, n, sizeof(double));
    const long long nz = nnz;
    put(out, &nz, 1, sizeof(long long));
    put(out, ptr, n + 1, sizeof(long));
    put(out, col, nnz, sizeof(long));
    put(out, coef, 4 * nnz, sizeof(double));
    put(out, point, 4 * nnz, sizeof(double));
    put(out, y, 2 * n, sizeof(double));
    put(out, b, 2 * n, sizeof(double));
    put(out, &esum, 1, sizeof(double));
    put(out, phi, na, sizeof(double));
    fclose(out);

    free(hdr); free(par); free(V); free(T); free(inc_ptr); free(inc_tri); free(ax); free(q);
    free(x); free(ta); free(tn); free(area); free(nn); free(rho2); free(rows); free(cnt);
    free(ptr); free(col); free(pp); free(coef); free(point); free(y); free(b); free(phi);
    return 0;
}

// Expansion bases of the FMM for the Laplace kernel 1/(4 pi r) and the
// screened-Coulomb kernel e^{-kappa r}/(4 pi r) (Section 2, Eq. 3; the four
// FMM calls of the Section 2 computation flow use these two kernels with
// charge and dipole sources).
//
// Real orthonormal spherical harmonics Y_nm (m = -n..n, index k = n^2+n+m)
// are generated as regular solid harmonics R_k(u) = |u|^n Y_nm(u/|u|) by the
// three-term recurrence of the associated Legendre functions in Cartesian
// form (no angles), starting from (x + i y)^m.
//
// Level-scaled bases at a level with box side s, u = v/s:
//   Laplace   regular  Reg_k(v) = R_k(u)
//             singular Sing_k(v) = R_k(u) / |u|^{2n+1}
//   screened  regular  Reg_k(v) = [g_n(kappa|v|) / g_n(kappa s)] R_k(u),
//                      g_n(x) = i_n(x)/x^n (i_n modified spherical Bessel,
//                      first kind, i_0 = sinh(x)/x), an entire function of x^2
//             singular Sing_k(v) = [k_n(kappa|v|) / k_n(kappa s)] R_k(u)/|u|^n,
//                      k_0 = e^{-x}/x
// Kernel expansions (|y-c| < |x-c|):
//   1/(4 pi |x-y|)            = sum_k Reg_k(y-c) Sing_k(x-c) / ((2n+1) s)
//   e^{-kappa|x-y|}/(4pi|x-y|)= sum_k Reg_k(y-c) Sing_k(x-c) kappa i_n(kappa s) k_n(kappa s)
//
// Every routine is templated on the scalar so that a dual number (value,
// directional derivative) yields dipole moments and normal derivatives.
#pragma once
#include <hip/hip_runtime.h>

namespace afmpb {

template <typename R>
struct Dual {
    R v, d;
    __device__ Dual() : v(0), d(0) {}
    __device__ Dual(R a) : v(a), d(0) {}
    __device__ Dual(R a, R b) : v(a), d(b) {}
};
template <typename R> __device__ inline Dual<R> operator+(Dual<R> a, Dual<R> b) { return {a.v + b.v, a.d + b.d}; }
template <typename R> __device__ inline Dual<R> operator-(Dual<R> a, Dual<R> b) { return {a.v - b.v, a.d - b.d}; }
template <typename R> __device__ inline Dual<R> operator*(Dual<R> a, Dual<R> b) { return {a.v * b.v, a.v * b.d + a.d * b.v}; }
template <typename R> __device__ inline Dual<R> operator*(R a, Dual<R> b) { return {a * b.v, a * b.d}; }
template <typename R> __device__ inline Dual<R> operator*(Dual<R> b, R a) { return {a * b.v, a * b.d}; }
template <typename R> __device__ inline Dual<R> operator/(Dual<R> a, R b) { return {a.v / b, a.d / b}; }

template <typename R> __device__ inline R val(R a) { return a; }
template <typename R> __device__ inline R val(Dual<R> a) { return a.v; }

// Emits (k, n, value) for every regular solid harmonic of degree <= P, in
// the order m = 0..P, n = m..P (for m > 0 the cosine entry k = n^2+n+m and
// the sine entry k = n^2+n-m).  norm[k] are the orthonormalisation factors;
// rec[2 (n (P+1) + m) + {0, 1}] = {(2n-1)/(n-m), (n+m-1)/(n-m)} are the
// recurrence coefficients (a table, so no division runs per point).
template <typename R, typename S, typename F, typename NT>
__device__ inline void for_each_regular(S x, S y, S z, int P, const NT *norm, const NT *rec,
                                        F &&emit) {
    S r2 = (x * x + y * y) + z * z;
    S cm(R(1)), sm(R(0));   // Re/Im of (x + i y)^m
    R dfact = R(1);         // (2m-1)!!
    for (int m = 0; m <= P; ++m) {
        S pc = cm * dfact, ps = sm * dfact;     // q_m^m
        S qc(R(0)), qs(R(0));                   // q_{m-1}^m = 0
        for (int n = m; n <= P; ++n) {
            if (n > m) {
                const NT *ab = rec + 2 * (n * (P + 1) + m);
                const R a = R(ab[0]), b = R(ab[1]);
                S nc = a * (z * pc) - b * (r2 * qc);
                S ns = a * (z * ps) - b * (r2 * qs);
                qc = pc; qs = ps;
                pc = nc; ps = ns;
            }
            int k0 = n * n + n;
            if (m == 0) {
                emit(k0, n, R(norm[k0]) * pc);
            } else {
                emit(k0 + m, n, R(norm[k0 + m]) * pc);
                emit(k0 - m, n, R(norm[k0 - m]) * ps);
            }
        }
        S c2 = cm * x - sm * y;
        sm = cm * y + sm * x;
        cm = c2;
        dfact *= R(2 * m + 1);
    }
}

// for_each_regular for a compile-time order P: the loops unroll completely,
// the recurrence coefficients become constants (the same double values the
// table holds, rounded to R) and every index is static.
template <int P, typename R, typename S, typename F, typename NT>
__device__ inline void for_each_regular_p(S x, S y, S z, const NT *norm, F &&emit) {
    S r2 = (x * x + y * y) + z * z;
    S cm(R(1)), sm(R(0));
    R dfact = R(1);
#pragma unroll
    for (int m = 0; m <= P; ++m) {
        S pc = cm * dfact, ps = sm * dfact;
        S qc(R(0)), qs(R(0));
#pragma unroll
        for (int n = m; n <= P; ++n) {
            if (n > m) {
                const R a = R((2.0 * n - 1.0) / (n - m)), b = R((n + m - 1.0) / (n - m));
                S nc = a * (z * pc) - b * (r2 * qc);
                S ns = a * (z * ps) - b * (r2 * qs);
                qc = pc; qs = ps;
                pc = nc; ps = ns;
            }
            const int k0 = n * n + n;
            if (m == 0) {
                emit(k0, n, R(norm[k0]) * pc);
            } else {
                emit(k0 + m, n, R(norm[k0 + m]) * pc);
                emit(k0 - m, n, R(norm[k0 - m]) * ps);
            }
        }
        S c2 = cm * x - sm * y;
        sm = cm * y + sm * x;
        cm = c2;
        dfact *= R(2 * m + 1);
    }
}

// for_each_regular_p without the orthonormalisation factors and restricted
// to the orders m = M0..M1: emits the raw solid harmonics (k, n, q) with
// R_k = norm[k] q, for a caller that applies the factors once to a sum over
// many points (and may split the orders m among several lanes).
template <int P, int M0, int M1, typename R, typename S, typename F>
__device__ inline void for_each_solid_p(S x, S y, S z, F &&emit) {
    S r2 = (x * x + y * y) + z * z;
    S cm(R(1)), sm(R(0));
    R dfact = R(1);
#pragma unroll
    for (int m = 0; m <= M1; ++m) {
        if (m >= M0) {
            S pc = cm * dfact, ps = sm * dfact;
            S qc(R(0)), qs(R(0));
#pragma unroll
            for (int n = m; n <= P; ++n) {
                if (n > m) {
                    const R a = R((2.0 * n - 1.0) / (n - m)), b = R((n + m - 1.0) / (n - m));
                    S nc = a * (z * pc) - b * (r2 * qc);
                    S ns = a * (z * ps) - b * (r2 * qs);
                    qc = pc; qs = ps;
                    pc = nc; ps = ns;
                }
                const int k0 = n * n + n;
                if (m == 0) {
                    emit(k0, n, pc);
                } else {
                    emit(k0 + m, n, pc);
                    emit(k0 - m, n, ps);
                }
            }
        }
        if (m < M1) {
            S c2 = cm * x - sm * y;
            sm = cm * y + sm * x;
            cm = c2;
            dfact *= R(2 * m + 1);
        }
    }
}

// Number of harmonics of orders m = M0..M1 up to degree P.
constexpr int solid_count(int P, int M0, int M1) {
    int c = 0;
    for (int m = M0; m <= M1; ++m) c += (m == 0 ? 1 : 2) * (P + 1 - m);
    return c;
}

// The first order h of the second of two ranges 0..h-1, h..P, chosen so that
// the larger of the two holds as few harmonics as possible.
constexpr int solid_split(int P) {
    int best = 1, bmax = 1 << 30;
    for (int h = 1; h <= P; ++h) {
        const int a = solid_count(P, 0, h - 1), b = solid_count(P, h, P);
        const int mx = a > b ? a : b;
        if (mx < bmax) { bmax = mx; best = h; }
    }
    return best;
}

// g_n(x) = i_n(x) / x^n for n = 0..P as functions of t = x^2: series for
// n = P and P-1, then the downward recurrence g_{n-1} = t g_{n+1} + (2n+1) g_n.
// inv_dfact[n] = 1/(2n+1)!!; ser[k] = 1/(2 k (2n+2k+1)) is the ratio of
// consecutive series terms over t (row 0: n = P, row 1: n = P-1).
constexpr int GSER = 200;

template <typename R, typename S, typename ST>
__device__ inline S g_series(int n, S t, const R *inv_dfact, const ST *ser) {
    S sum(R(1)), term(R(1));
    for (int k = 1; k < GSER; ++k) {
        term = term * t * R(ser[k]);
        sum = sum + term;
        R tv = val(term), sv = val(sum);
        if ((tv < R(0) ? -tv : tv) <= R(1e-17) * (sv < R(0) ? -sv : sv)) break;
    }
    return sum * inv_dfact[n];
}

template <typename R, typename S, typename ST>
__device__ inline void g_all(int P, S t, const R *inv_dfact, const ST *ser, S *g) {
    g[P] = g_series<R, S>(P, t, inv_dfact, ser);
    if (P >= 1) g[P - 1] = g_series<R, S>(P - 1, t, inv_dfact, ser + GSER);
    for (int n = P - 1; n >= 1; --n) g[n - 1] = t * g[n + 1] + R(2 * n + 1) * g[n];
}

// g_all for a compile-time order (static indices: g stays in registers).
template <int P, typename R, typename S, typename ST>
__device__ inline void g_all_p(S t, const R *inv_dfact, const ST *ser, S *g) {
    g[P] = g_series<R, S>(P, t, inv_dfact, ser);
    if (P >= 1) g[P - 1] = g_series<R, S>(P - 1, t, inv_dfact, ser + GSER);
#pragma unroll
    for (int n = P - 1; n >= 1; --n) g[n - 1] = t * g[n + 1] + R(2 * n + 1) * g[n];
}

}  // namespace afmpb

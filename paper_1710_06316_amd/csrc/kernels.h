// Point kernels of the boundary-integral equation (Section 2, Eq. 3) and the
// four integrands of the patch coefficients (Eq. 6), for double and float.
//
// R = x - y with x the target node p (normal n_p = n0) and y the source point
// on patch t (normal n_t = n).  G = 1/(4 pi r), u = e^{-kappa r}/(4 pi r).
//   A-integrand  G - u                         = -expm1(-s)/(4 pi r)
//   B-integrand  dG/dn/ebar - du/dn            = (R.n)/(4 pi r^3) (1/ebar - e(1+s))
//   C-integrand  dG/dn0 - du/dn0/ebar          = -(R.n0)/(4 pi r^3) (1 - e(1+s)/ebar)
//   D-integrand  (d2G/dn0dn - d2u/dn0dn)/ebar  = [(n0.n) a(s)/r^3 - (R.n0)(R.n) b(s)/r^5]
//                                                / (4 pi ebar)
// with s = kappa r, e = e^{-s}, a(s) = 1 - e(1+s), b(s) = 3 - e(3+3s+s^2).
// a is taken from its Taylor series below s = 0.1 and from 1 - e - s e above
// (1 - e from expm1 below s = 0.5), and b = 3 a - s^2 e, so the
// Laplace/screened difference never cancels.
#pragma once
#include <hip/hip_runtime.h>

namespace afmpb {

constexpr double INV_4PI = 0.079577471545947667884441881686257181;

// Taylor coefficients: a(s) = sum_{k>=2} (-1)^k (k-1) s^k/k!.
struct DiffSeries {
    double a[11];
    constexpr DiffSeries() : a() {
        double fact = 1.0;
        for (int k = 1; k <= 10; ++k) {
            fact *= k;
            double sg = (k & 1) ? -1.0 : 1.0;
            a[k] = (k >= 2) ? sg * (k - 1) / fact : 0.0;
        }
    }
};

template <typename R>
__device__ inline void diff_factors(R s, R e, R em1, R &fa, R &fb) {
    constexpr DiffSeries S;
    if (s < R(0.1)) {
        R pa = R(S.a[10]);
#pragma unroll
        for (int k = 9; k >= 2; --k) pa = pa * s + R(S.a[k]);
        fa = pa * s * s;
    } else {
        fa = em1 - s * e;                    // 1 - e - s e
    }
    // b = 3 a - s^2 e: the two terms cancel to about a third of 3 a as s -> 0
    // (both a and b ~ s^2/2), so b keeps a relative error of a few times a's
    fb = R(3) * fa - (s * s) * e;
}

// 1/sqrt(x) for x > 0: the hardware estimate refined by Newton's method for
// the root of y^-2 - x (each step y += y (1 - x y^2) / 2 about doubles the
// correct bits; two steps from the double-precision estimate, one correction
// of the residual's second order in the last).
__device__ inline double inv_sqrt(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    y = fma(y * e, 0.5, y);
    e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}
__device__ inline float inv_sqrt(float x) { return 1.0f / sqrtf(x); }

// The four integrands (without the patch area / quadrature weight).
template <typename R>
struct Abcd {
    R A, B, C, D;
};

template <typename R>
__device__ inline Abcd<R> abcd_point(R rx, R ry, R rz, R n0x, R n0y, R n0z, R nx, R ny,
                                     R nz, R kappa, R inv_ebar) {
    R r2 = (rx * rx + ry * ry) + rz * rz;
    R ir = inv_sqrt(r2);
    R r = r2 * ir;
    R ir3 = ir * ir * ir;
    R s = kappa * r;
    R e = exp(-s);
    // 1 - e: from expm1 while e is close to 1, else the plain difference
    // (which loses no digits once e < e^-0.5)
    R em1;
    if (s < R(0.5)) em1 = -expm1(-s);
    else em1 = R(1) - e;
    R Rn = (rx * nx + ry * ny) + rz * nz;
    R Rn0 = (rx * n0x + ry * n0y) + rz * n0z;
    R n0n = (n0x * nx + n0y * ny) + n0z * nz;
    R fa, fb;
    diff_factors(s, e, em1, fa, fb);
    R e1 = e * (R(1) + s);
    Abcd<R> o;
    o.A = em1 * ir * R(INV_4PI);
    o.B = Rn * ir3 * R(INV_4PI) * (inv_ebar - e1);
    o.C = -Rn0 * ir3 * R(INV_4PI) * (R(1) - e1 * inv_ebar);
    o.D = (n0n * fa * ir3 - Rn0 * Rn * fb * ir3 * ir * ir) * R(INV_4PI) * inv_ebar;
    return o;
}

}  // namespace afmpb

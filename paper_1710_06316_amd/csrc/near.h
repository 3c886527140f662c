// Near set (CSR over Morton-ordered rows) with patch-minus-point corrections.
#pragma once
#include "geometry.h"

namespace afmpb {

struct NearSet {
    DBuf<long long> ptr;     // [n+1]
    DBuf<int> col;           // [nnz] ascending per row, Morton positions
    DBuf<double> delta;      // [nnz][4] corrections of {A, B, C, D}
    DBuf<float> delta32;     // the same, rounded to FP32 (mixed-precision matvec)
    DBuf<double> rule;       // quadrature rule table of the correction kernel
    long long nnz = 0;
};

// The near set (ptr, col) on stream s; returns with s drained.
void build_near(const NodeSoA &nd, long long n, double eta, NearSet &out, hipStream_t s);

// The corrections (delta, delta32) of a built near set, enqueued on stream s
// without waiting for them: the caller orders later uses after s.
void near_coeffs(const NodeSoA &nd, long long n, const double *V, const int *T,
                 const double *tri_n, const int *inc_ptr, const int *inc_tri, const int *perm,
                 double kappa, double ebar, NearSet &out, hipStream_t s);

}  // namespace afmpb

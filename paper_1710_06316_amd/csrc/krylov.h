// FP64 vector kernels of the Krylov solver, right-hand side and energy.
#pragma once
#include "geometry.h"

namespace afmpb {

// Scratch elements dots() needs for nvec vectors of length len (size the
// scratch once for the largest nvec: dots() grows it otherwise).
long long dots_scratch(long long len, int nvec);
// out[j] = <V[j], w> for j < nvec (V rows of length len, stride ld).
void dots(const double *V, long long ld, int nvec, const double *w, long long len, double *out,
          DBuf<double> &scratch, hipStream_t s);
// w += sign * V^T c
void gemv(const double *V, long long ld, int nvec, const double *c, double sign, long long len,
          double *w, hipStream_t s);
void scale(const double *a, double alpha, long long len, double *out, hipStream_t s);
void axpby(double a, const double *x, double b, const double *y, long long len, double *out,
           hipStream_t s);
void rhs(const NodeSoA &nd, long long n, const double *ax, const double *q, long long na,
         double eps_s, double *b, hipStream_t s);
void reaction_potential(const NodeSoA &nd, long long n, const double *x, const double *ax,
                        long long na, double ebar, double *phi, hipStream_t s);

}  // namespace afmpb

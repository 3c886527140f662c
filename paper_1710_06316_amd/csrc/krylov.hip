// FP64 Krylov kernels (Section 3.4: restarted GMRES; the FMM input is the
// last basis vector itself), right-hand side of Eq. (5) and the reaction
// potential at the atoms.
#include "krylov.h"
#include "kernels.h"

namespace afmpb {

namespace {

constexpr int DOT_BLOCK = 256;
constexpr int DOT_CHUNK = DOT_BLOCK * 16;

__device__ inline double block_sum(double v) {
    __shared__ double ws[DOT_BLOCK / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) ws[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < DOT_BLOCK / 64; ++w) t += ws[w];
    __syncthreads();
    return t;
}

// partial[j][blk] = sum over the block's chunk of V[j][k] * w[k]
__global__ void k_dots_partial(const double *__restrict__ V, long long ld,
                               const double *__restrict__ w, long long len, int nblk,
                               double *__restrict__ partial) {
    const int blk = blockIdx.x, j = blockIdx.y;
    const double *v = V + (long long)j * ld;
    long long b = (long long)blk * DOT_CHUNK;
    double s = 0.0;
    for (int i = 0; i < 16; ++i) {
        long long k = b + (long long)i * DOT_BLOCK + threadIdx.x;
        if (k < len) s += v[k] * w[k];
    }
    s = block_sum(s);
    if (threadIdx.x == 0) partial[(long long)j * nblk + blk] = s;
}

__global__ void k_dots_final(const double *__restrict__ partial, int nblk, int nvec,
                             double *__restrict__ out) {
    int j = blockIdx.x;
    if (j >= nvec) return;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += partial[(long long)j * nblk + b];
    s = block_sum(s);
    if (threadIdx.x == 0) out[j] = s;
}

// w[k] += sign * sum_j V[j][k] c[j]
__global__ void k_gemv(const double *__restrict__ V, long long ld, int nvec,
                       const double *__restrict__ c, double sign, long long len,
                       double *__restrict__ w) {
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= len) return;
    double s = 0.0;
    for (int j = 0; j < nvec; ++j) s += V[(long long)j * ld + k] * c[j];
    w[k] += sign * s;
}

__global__ void k_scale(const double *__restrict__ a, double alpha, long long len,
                        double *__restrict__ out) {
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < len) out[k] = alpha * a[k];
}

__global__ void k_axpby(double a, const double *__restrict__ x, double b,
                        const double *__restrict__ y, long long len, double *__restrict__ out) {
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < len) out[k] = a * x[k] + b * y[k];
}

// b_f(p) = (1/eps_s) sum_k q_k G(p,k), b_h(p) = (1/eps_s) sum_k q_k dG(p,k)/dn_p
__global__ void k_rhs(NodeSoA nd, long long n, const double *__restrict__ ax,
                      const double *__restrict__ q, long long na, double inv_eps, double *b) {
    __shared__ double A[4][256];
    long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    bool act = p < n;
    double x = act ? nd.x[p] : 0, y = act ? nd.y[p] : 0, z = act ? nd.z[p] : 0;
    double nx = act ? nd.nx[p] : 0, ny = act ? nd.ny[p] : 0, nz = act ? nd.nz[p] : 0;
    double sf = 0.0, sh = 0.0;
    for (long long a0 = 0; a0 < na; a0 += 256) {
        long long a = a0 + threadIdx.x;
        __syncthreads();
        if (a < na) {
            A[0][threadIdx.x] = ax[3 * a]; A[1][threadIdx.x] = ax[3 * a + 1];
            A[2][threadIdx.x] = ax[3 * a + 2]; A[3][threadIdx.x] = q[a];
        }
        __syncthreads();
        int cnt = (int)min(256ll, na - a0);
        if (act)
            for (int j = 0; j < cnt; ++j) {
                double rx = x - A[0][j], ry = y - A[1][j], rz = z - A[2][j];
                double r2 = (rx * rx + ry * ry) + rz * rz;
                double ir = 1.0 / sqrt(r2);
                double Rn = (rx * nx + ry * ny) + rz * nz;
                sf += A[3][j] * ir;
                sh -= A[3][j] * Rn * ir * ir * ir;
            }
    }
    if (act) {
        b[p] = sf * INV_4PI * inv_eps;
        b[n + p] = sh * INV_4PI * inv_eps;
    }
}

// phi_reac(r_k) = sum_t a_t [ebar h_t G(r_k, r_t) - f_t dG(r_k, r_t)/dn_t]
__global__ void k_reaction(NodeSoA nd, long long n, const double *__restrict__ x,
                           const double *__restrict__ ax, long long na, double ebar,
                           double *__restrict__ phi) {
    __shared__ double S[8][256];
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    bool act = k < na;
    double px = act ? ax[3 * k] : 0, py = act ? ax[3 * k + 1] : 0, pz = act ? ax[3 * k + 2] : 0;
    double s = 0.0;
    for (long long t0 = 0; t0 < n; t0 += 256) {
        long long t = t0 + threadIdx.x;
        __syncthreads();
        if (t < n) {
            S[0][threadIdx.x] = nd.x[t]; S[1][threadIdx.x] = nd.y[t]; S[2][threadIdx.x] = nd.z[t];
            S[3][threadIdx.x] = nd.nx[t]; S[4][threadIdx.x] = nd.ny[t]; S[5][threadIdx.x] = nd.nz[t];
            S[6][threadIdx.x] = nd.area[t] * x[t];
            S[7][threadIdx.x] = nd.area[t] * x[n + t];
        }
        __syncthreads();
        int cnt = (int)min(256ll, n - t0);
        if (act)
            for (int j = 0; j < cnt; ++j) {
                double rx = px - S[0][j], ry = py - S[1][j], rz = pz - S[2][j];
                double r2 = (rx * rx + ry * ry) + rz * rz;
                double ir = 1.0 / sqrt(r2);
                double Rn = (rx * S[3][j] + ry * S[4][j]) + rz * S[5][j];
                s += ebar * S[7][j] * ir - S[6][j] * Rn * ir * ir * ir;
            }
    }
    if (act) phi[k] = s * INV_4PI;
}

}  // namespace

long long dots_scratch(long long len, int nvec) {
    return ((len + DOT_CHUNK - 1) / DOT_CHUNK) * (long long)nvec;
}

void dots(const double *V, long long ld, int nvec, const double *w, long long len, double *out,
          DBuf<double> &scratch, hipStream_t s) {
    int nblk = (int)((len + DOT_CHUNK - 1) / DOT_CHUNK);
    if (scratch.n < (size_t)nblk * nvec) scratch.alloc((size_t)nblk * nvec);
    k_dots_partial<<<dim3(nblk, nvec), DOT_BLOCK, 0, s>>>(V, ld, w, len, nblk, scratch.p);
    KCHK();
    k_dots_final<<<nvec, DOT_BLOCK, 0, s>>>(scratch.p, nblk, nvec, out);
    KCHK();
}

void gemv(const double *V, long long ld, int nvec, const double *c, double sign, long long len,
          double *w, hipStream_t s) {
    k_gemv<<<grid_for(len, 256), 256, 0, s>>>(V, ld, nvec, c, sign, len, w);
    KCHK();
}

void scale(const double *a, double alpha, long long len, double *out, hipStream_t s) {
    k_scale<<<grid_for(len, 256), 256, 0, s>>>(a, alpha, len, out);
    KCHK();
}

void axpby(double a, const double *x, double b, const double *y, long long len, double *out,
           hipStream_t s) {
    k_axpby<<<grid_for(len, 256), 256, 0, s>>>(a, x, b, y, len, out);
    KCHK();
}

void rhs(const NodeSoA &nd, long long n, const double *ax, const double *q, long long na,
         double eps_s, double *b, hipStream_t s) {
    k_rhs<<<grid_for(n, 256), 256, 0, s>>>(nd, n, ax, q, na, 1.0 / eps_s, b);
    KCHK();
}

void reaction_potential(const NodeSoA &nd, long long n, const double *x, const double *ax,
                        long long na, double ebar, double *phi, hipStream_t s) {
    if (na == 0) return;
    k_reaction<<<grid_for(na, 256), 256, 0, s>>>(nd, n, x, ax, na, ebar, phi);
    KCHK();
}

}  // namespace afmpb

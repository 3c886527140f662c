// Far field of the node-patch matvec (Section 2 computation flow, step 3b:
// the single/double-layer Laplace and screened-Coulomb FMM evaluations, done
// together in one traversal as the paper's ViewSet does, Section 3.1).
//
// Sources per node t: charge sigma_t = a_t h_t for both kernels, dipole
// -a_t f_t n_t / ebar for the Laplace expansion and -a_t f_t n_t for the
// screened one; targets: potential and normal derivative at every node.
//
// Translation operators are dense K x K matrices, one per (level, offset
// class) for M2L and per (level, child octant) for M2M/L2L, obtained by
// projecting the translated basis functions onto spherical harmonics with a
// Gauss-Legendre x trapezoid product rule on a sphere and one batched GEMM.
#include <algorithm>
#include <cmath>

#include "basis.h"
#include "fmm.h"
#include "prof.h"

namespace afmpb {

void gauss_legendre01(int nq, double *x, double *w);

namespace {

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Regular level-scaled basis of kernel `kern` at v (box side s, level lev).
template <typename R, typename S, typename F>
__device__ inline void regular_basis(const BasisDev &B, int kern, int lev, S vx, S vy, S vz,
                                     F &&emit) {
    const R is = R(1.0 / B.side[lev]);
    S ux = vx * is, uy = vy * is, uz = vz * is;
    if (kern == 0 || !B.screened) {
        for_each_regular<R>(ux, uy, uz, B.P, B.norm, B.rec, [&](int k, int, S r) { emit(k, r); });
    } else {
        R ks = R(B.kappa * B.side[lev]);
        S t = (ks * ks) * ((ux * ux + uy * uy) + uz * uz);
        S g[MAXP + 1];
        R inv_df[MAXP + 2];
        for (int n = 0; n <= B.P + 1; ++n) inv_df[n] = R(B.inv_dfact[n]);
        g_all<R, S>(B.P, t, inv_df, B.gser, g);
        const double *gi = B.ginv + (long long)lev * (B.P + 1);
        for_each_regular<R>(ux, uy, uz, B.P, B.norm, B.rec,
                            [&](int k, int n, S r) { emit(k, r * (g[n] * R(gi[n]))); });
    }
}

// Recurrence tables of the expansion bases in the working precision, staged
// in LDS by the point kernels (P2M, L2P), so that each use is an LDS read
// rather than a memory load on the recurrence's critical path.  Values are
// those of the tables in memory, rounded to R once.
template <typename R>
struct BasisTab {
    const R *rec, *norm, *ginv, *idf, *ser;
};

// LDS bytes of the staged tables for order P and nlev tree levels.
__host__ __device__ inline size_t basis_tab_bytes(int P, int nlev, size_t elem) {
    const size_t K = (size_t)(P + 1) * (P + 1);
    return (3 * K + (size_t)nlev * (P + 1) + (P + 2) + 2 * GSER) * elem;
}

// Block-cooperative copy of the tables into dynamic LDS at `raw`; ends with a
// block barrier.
template <typename R>
__device__ inline BasisTab<R> stage_basis(const BasisDev &B, int nlev, unsigned char *raw) {
    const int P = B.P, K = B.K;
    R *rec = reinterpret_cast<R *>(raw);
    R *norm = rec + 2 * K, *ginv = norm + K, *idf = ginv + nlev * (P + 1), *ser = idf + P + 2;
    for (int i = threadIdx.x; i < 2 * K; i += blockDim.x) rec[i] = R(B.rec[i]);
    for (int i = threadIdx.x; i < K; i += blockDim.x) norm[i] = R(B.norm[i]);
    for (int i = threadIdx.x; i < nlev * (P + 1); i += blockDim.x) ginv[i] = R(B.ginv[i]);
    for (int i = threadIdx.x; i < P + 2; i += blockDim.x) idf[i] = R(B.inv_dfact[i]);
    if (B.screened)
        for (int i = threadIdx.x; i < 2 * GSER; i += blockDim.x) ser[i] = R(B.gser[i]);
    __syncthreads();
    return BasisTab<R>{rec, norm, ginv, idf, ser};
}

// regular_basis with the staged tables (same values, same order of operations).
template <typename R, typename S, typename F>
__device__ inline void regular_basis_tab(const BasisDev &B, const BasisTab<R> &T, int kern,
                                         int lev, S vx, S vy, S vz, F &&emit) {
    const R is = R(1.0 / B.side[lev]);
    S ux = vx * is, uy = vy * is, uz = vz * is;
    if (kern == 0 || !B.screened) {
        for_each_regular<R>(ux, uy, uz, B.P, T.norm, T.rec, [&](int k, int, S r) { emit(k, r); });
    } else {
        R ks = R(B.kappa * B.side[lev]);
        S t = (ks * ks) * ((ux * ux + uy * uy) + uz * uz);
        S g[MAXP + 1];
        g_all<R, S>(B.P, t, T.idf, T.ser, g);
        const R *gi = T.ginv + lev * (B.P + 1);
        for_each_regular<R>(ux, uy, uz, B.P, T.norm, T.rec,
                            [&](int k, int n, S r) { emit(k, r * (g[n] * gi[n])); });
    }
}

// The same for a compile-time order PC (PC = 0: B.P at run time).
template <int PC, typename R, typename S, typename F>
__device__ inline void regular_basis_o(const BasisDev &B, const BasisTab<R> &T, int kern,
                                       int lev, S vx, S vy, S vz, F &&emit) {
    if constexpr (PC == 0) {
        regular_basis_tab<R, S>(B, T, kern, lev, vx, vy, vz, emit);
    } else {
        const R is = R(1.0 / B.side[lev]);
        S ux = vx * is, uy = vy * is, uz = vz * is;
        if (kern == 0 || !B.screened) {
            for_each_regular_p<PC, R>(ux, uy, uz, T.norm, [&](int k, int, S r) { emit(k, r); });
        } else {
            R ks = R(B.kappa * B.side[lev]);
            S t = (ks * ks) * ((ux * ux + uy * uy) + uz * uz);
            S g[PC + 1];
            g_all_p<PC, R, S>(t, T.idf, T.ser, g);
            const R *gi = T.ginv + lev * (PC + 1);
            for_each_regular_p<PC, R>(ux, uy, uz, T.norm,
                                      [&](int k, int n, S r) { emit(k, r * (g[n] * gi[n])); });
        }
    }
}

// ------------------------- operator construction ---------------------------

struct MatDesc {
    int kind;          // 0: M2L (singular source basis), 1: M2M/L2L (regular)
    int kern, lev;     // kernel, basis level (M2L: box level; M2M: parent level)
    double dx, dy, dz; // centre of the evaluation sphere relative to the basis origin
    double rq;         // sphere radius
    long long dst;     // offset of the K x K output
};

// Per-level constants: 1/g_n(kappa s), 1/k_n(kappa s) and the expansion
// weights W_n (Laplace: 1/((2n+1) s); screened: kappa i_n(ks) k_n(ks)).
__global__ void k_level_consts(BasisDev B, int nlev, double *ginv, double *kinv, double *W) {
    int lev = blockIdx.x;
    if (lev >= nlev || threadIdx.x != 0) return;
    const int P = B.P;
    const double s = B.side[lev];
    for (int n = 0; n <= P; ++n) W[(0 * 64 + lev) * (P + 1) + n] = 1.0 / ((2.0 * n + 1.0) * s);
    if (!B.screened) {
        for (int n = 0; n <= P; ++n) {
            ginv[lev * (P + 1) + n] = 1.0;
            kinv[lev * (P + 1) + n] = 1.0;
            W[(1 * 64 + lev) * (P + 1) + n] = 1.0 / ((2.0 * n + 1.0) * s);
        }
        return;
    }
    const double ks = B.kappa * s;
    double g[MAXP + 1], kn[MAXP + 2];
    g_all<double, double>(P, ks * ks, B.inv_dfact, B.gser, g);
    kn[0] = exp(-ks) / ks;
    kn[1] = exp(-ks) * (1.0 + ks) / (ks * ks);
    for (int n = 1; n < P; ++n) kn[n + 1] = kn[n - 1] + (2.0 * n + 1.0) / ks * kn[n];
    for (int n = 0; n <= P; ++n) {
        ginv[lev * (P + 1) + n] = 1.0 / g[n];
        kinv[lev * (P + 1) + n] = 1.0 / kn[n];
        W[(1 * 64 + lev) * (P + 1) + n] = B.kappa * (g[n] * pow(ks, (double)n)) * kn[n];
    }
}

// Yw[q][k] = w_q Y_k(s_q) on the unit sphere.
__global__ void k_sphere_table(BasisDev B, int Q, const double *dir, const double *wq,
                               double *Yw) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q) return;
    double x = dir[3 * q], y = dir[3 * q + 1], z = dir[3 * q + 2], w = wq[q];
    const int K = B.K;
    for_each_regular<double>(x, y, z, B.P, B.norm, B.rec,
                             [&](int k, int, double r) { Yw[(long long)q * K + k] = w * r; });
}

// B[m][q][j]: basis values of matrix m at quadrature point q, and row scales.
__global__ void k_basis_samples(BasisDev B, const MatDesc *desc, int nmat, int Q,
                                const double *dir, const double *kinv, const double *W,
                                double *out, double *rowscale, int nlev) {
    extern __shared__ __align__(16) unsigned char tab_raw[];
    const BasisTab<double> tab = stage_basis<double>(B, nlev, tab_raw);
    long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long long)nmat * Q) return;
    int m = (int)(id / Q), q = (int)(id % Q);
    const MatDesc d = desc[m];
    const int K = B.K, P = B.P;
    const double s = B.side[d.lev];
    double vx = d.dx + d.rq * dir[3 * q], vy = d.dy + d.rq * dir[3 * q + 1],
           vz = d.dz + d.rq * dir[3 * q + 2];
    double *o = out + id * K;
    if (d.kind == 1) {
        regular_basis_tab<double, double>(B, tab, d.kern, d.lev, vx, vy, vz,
                                          [&](int k, double r) { o[k] = r; });
    } else {
        double ux = vx / s, uy = vy / s, uz = vz / s;
        double ru = sqrt((ux * ux + uy * uy) + uz * uz);
        const double *Wl = W + ((long long)d.kern * 64 + d.lev) * (P + 1);
        double rad[MAXP + 1];
        if (d.kern == 0 || !B.screened) {
            double ir = 1.0 / ru, f = ir;
            for (int n = 0; n <= P; ++n) { rad[n] = f * Wl[n]; f *= ir * ir; }
        } else {
            double x = B.kappa * s * ru;
            double k0 = exp(-x) / x, k1 = exp(-x) * (1.0 + x) / (x * x);
            double km = k0, kc = k1, ir = 1.0 / ru, f = 1.0;
            const double *ki = kinv + (long long)d.lev * (P + 1);
            for (int n = 0; n <= P; ++n) {
                double kn;
                if (n == 0) kn = k0;
                else if (n == 1) kn = k1;
                else { double nx = km + (2.0 * (n - 1) + 1.0) / x * kc; km = kc; kc = nx; kn = kc; }
                rad[n] = kn * ki[n] * f * Wl[n];
                f *= ir;
            }
        }
        for_each_regular<double>(ux, uy, uz, P, tab.norm, tab.rec,
                                 [&](int k, int n, double r) { o[k] = r * rad[n]; });
    }
    if (q == 0) {
        // row scale 1/rho_n(rq) of the local basis (M2L only)
        double g[MAXP + 1];
        const bool scr = d.kind == 0 && d.kern == 1 && B.screened;
        if (scr) g_all<double, double>(P, (B.kappa * d.rq) * (B.kappa * d.rq), B.inv_dfact, B.gser, g);
        for (int n = 0; n <= P; ++n) {
            double sc = 1.0;
            if (d.kind == 0) {
                sc = 1.0 / pow(d.rq / s, (double)n);
                if (scr) sc *= 1.0 / (g[n] * B.ginv[(long long)d.lev * (P + 1) + n]);
            }
            for (int mm = -n; mm <= n; ++mm) rowscale[(long long)m * K + n * n + n + mm] = sc;
        }
    }
}

// C[m][i][j] = rs[m][i] * sum_q A[q][i] Bm[m][q][j]: 64 x 64 output tiles, 16 x 16
// threads with 4 x 4 outputs each (rows ty + 16 a, columns tx + 16 b), q in
// chunks of 16 through LDS (each output summed in q order).
__global__ void __launch_bounds__(256) k_project_gemm(const double *A, const double *Bm,
                                                      const double *rs, const MatDesc *desc,
                                                      int K, int Q, double *Tbase,
                                                      double *Ubase) {
    __shared__ double As[16][64], Bs[16][64];
    const int m = blockIdx.z;
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * 16 + tx;
    const double *B = Bm + (long long)m * Q * K;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int q0 = 0; q0 < Q; q0 += 16) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = tid + 256 * r, qq = e >> 6, ii = e & 63, q = q0 + qq;
            As[qq][ii] = (q < Q && i0 + ii < K) ? A[(long long)q * K + i0 + ii] : 0.0;
            Bs[qq][ii] = (q < Q && j0 + ii < K) ? B[(long long)q * K + j0 + ii] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            double av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = As[kk][ty + 16 * a];
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = Bs[kk][tx + 16 * b];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] += av[a] * bv[b];
        }
        __syncthreads();
    }
    double *C = desc[m].kind == 0 ? Tbase : Ubase;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int i = i0 + ty + 16 * a;
        if (i >= K) continue;
        const double sc = rs[(long long)m * K + i];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int j = j0 + tx + 16 * b;
            if (j < K) C[desc[m].dst + (long long)i * K + j] = sc * acc[a][b];
        }
    }
}

// packed[m][rt][ks][l] = A_m[16 rt + l % 16][4 ks + l / 16], A_m = op_m or its
// transpose, zero outside K x K.
__global__ void k_pack(const double *__restrict__ src, long long nmat, int K, int KK, int NRT,
                       int transpose, double *__restrict__ dst, float *__restrict__ dst32) {
    const long long PM = (long long)NRT * 16 * KK;
    long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nmat * PM) return;
    const long long m = id / PM;
    const long long r = id % PM;
    const int l = (int)(r % 64);
    const long long tk = r / 64;
    const int ks = (int)(tk % (KK / 4)), rt = (int)(tk / (KK / 4));
    const int row = rt * 16 + (l & 15), k = ks * 4 + (l >> 4);
    double v = 0.0;
    if (row < K && k < K)
        v = transpose ? src[m * K * K + (long long)k * K + row] : src[m * K * K + (long long)row * K + k];
    dst[id] = v;
    dst32[id] = (float)v;
}

__global__ void k_scale_copy(const double *__restrict__ a, double f, long long n,
                             double *__restrict__ b) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i] * f;
}

__global__ void k_to_float(const double *a, float *b, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}


// ------------------------------ far field ----------------------------------

struct TreeDev {
    const int *level, *parent, *cb, *nc, *ptb, *pte;
    const unsigned long long *prefix;
    const double *center;
};

// P2M / L2P work item: up to 4 leaves (consecutive in point order) with at
// most 64 points together share one wave, point q of the item on lane q; a
// leaf of more than 64 points is an item of its own, taken 64 points at a time.
// 16x16x4 matrix instructions (FP32 and FP64 accumulate in four result
// registers per lane; the operand layout is described with the batched
// translations below).
typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
template <typename R> struct Acc4;
template <> struct Acc4<double> { typedef d4v T; };
template <> struct Acc4<float> { typedef f4v T; };

__device__ inline d4v mfma16(double a, double b, d4v c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4v mfma16(float a, float b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// output row (within the 16-row tile) of result register r
template <typename R> __device__ inline int drow(int lane, int r);
template <> __device__ inline int drow<double>(int lane, int r) { return (lane >> 4) + 4 * r; }
template <> __device__ inline int drow<float>(int lane, int r) { return 4 * (lane >> 4) + r; }

struct PmItem {
    int first, cnt, tot;
    int offs[5];                 // point offset of each leaf in the item
    __device__ PmItem(const int *pm_leaf, const int *pm_first, const int *pm_count,
                      const TreeDev &T, int w) {
        first = pm_first[w];
        cnt = pm_count[w];
        offs[0] = 0;
        for (int g = 0; g < 4; ++g) {
            const int L = g < cnt ? pm_leaf[first + g] : -1;
            offs[g + 1] = offs[g] + (L >= 0 ? T.pte[L] - T.ptb[L] : 0);
        }
        tot = offs[cnt];
    }
    __device__ int leaf_of(int q) const {     // item point q -> leaf slot g
        return (q >= offs[1] && cnt > 1) + (q >= offs[2] && cnt > 2) + (q >= offs[3] && cnt > 3);
    }
};

// P2M: one block per item; wave w computes the expansions of kernel w % 2
// over the 64-point chunks c = w / 2, w / 2 + NCH, ... of the item.  Each
// lane evaluates the regular basis at one source point (about its own
// leaf's centre); the coefficients are emitted 16 at a time into LDS
// (W[slot][point]), and the per-leaf sums over points are one product on the
// matrix cores: W (16 x 64) times the 0/1 indicator of point-in-leaf
// (64 x 4, padded to 16 columns), 16 k-steps of four points.  The products
// by 1 and 0 are exact.  An item of one chunk writes M directly; a larger
// leaf (several chunks) sums its chunks' partial expansions in chunk order
// after a barrier (deterministic, the order of a serial pass).
template <typename R, int NCH>
__global__ void __launch_bounds__(128 * NCH) k_p2m(BasisDev B, TreeDev T, const int *pm_leaf,
                                                   const int *pm_first, const int *pm_count,
                                                   const R *px, const R *py, const R *pz,
                                                   const R *pnx, const R *pny, const R *pnz,
                                                   const R *sf, const R *sh, R inv_ebar, R *M,
                                                   int nlev) {
    __shared__ R Wv[NCH][2][16][65];
    __shared__ int kslot[NCH][2][16];
    extern __shared__ __align__(16) unsigned char tab_raw[];
    const BasisTab<R> tab = stage_basis<R>(B, nlev, tab_raw);
    // partial expansions of the chunks [NCH][2][K], after the basis tables
    R *part = reinterpret_cast<R *>(tab_raw + basis_tab_bytes(B.P, nlev, sizeof(R)));
    const PmItem it(pm_leaf, pm_first, pm_count, T, blockIdx.x);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int kern = wave & 1, ch = wave >> 1;
    const int K = B.K;
    const bool multi = it.tot > 64;                    // uniform for the block
    R (*W)[65] = Wv[ch][kern];
    int *ks_slot = kslot[ch][kern];
    for (int c0 = 64 * ch; c0 < it.tot; c0 += 64 * NCH) {
        const int q = c0 + lane;
        const bool ok = q < it.tot;
        const int g = it.leaf_of(ok ? q : 0);
        const int leaf = pm_leaf[it.first + g];
        const int lev = T.level[leaf];
        const int i = T.ptb[leaf] + (ok ? q - it.offs[g] : 0);
        const R cx = R(T.center[3 * leaf]), cy = R(T.center[3 * leaf + 1]);
        const R cz = R(T.center[3 * leaf + 2]);
        const R vx = ok ? px[i] - cx : R(0), vy = ok ? py[i] - cy : R(0), vz = ok ? pz[i] - cz : R(0);
        const R nx = ok ? pnx[i] : R(0), ny = ok ? pny[i] : R(0), nz = ok ? pnz[i] : R(0);
        const R qv = ok ? sh[i] : R(0);
        const R dmag = ok ? -sf[i] : R(0);
        const R dip = (kern == 0) ? dmag * inv_ebar : dmag;
        int cnt = 0;                       // coefficients emitted so far (uniform)
        auto flush = [&](int nslot) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // A[i][k] = W[i][4 ks + k] (i = lane % 16, k = lane / 16);
            // B[k][j] = 1 when point 4 ks + k of the chunk is in leaf j
            const int j = lane & 15, kq = lane >> 4;
            const int lo = j < it.cnt ? it.offs[j] - c0 : 0;
            const int hi = j < it.cnt ? it.offs[j + 1] - c0 : 0;
            typename Acc4<R>::T acc{0, 0, 0, 0};
#pragma unroll
            for (int ks = 0; ks < 16; ++ks) {
                const int pt = 4 * ks + kq;
                acc = mfma16(W[j][pt], (pt >= lo && pt < hi) ? R(1) : R(0), acc);
            }
            // D[i][j]: the sum of slot i over the points of leaf j
            if (j < it.cnt && max(lo, 0) < min(hi, 64)) {
                const int lg = pm_leaf[it.first + j];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int slot = drow<R>(lane, r);
                    if (slot < nslot) {
                        const int k = ks_slot[slot];
                        if (multi) {                     // one leaf (j = 0): this wave's partial
                            R *pk = part + (ch * 2 + kern) * K + k;
                            *pk = (c0 == 64 * ch) ? acc[r] : *pk + acc[r];
                        } else if (T.level[lg] >= 2) {
                            M[((long long)lg * 2 + kern) * K + k] = acc[r];
                        }
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        };
        regular_basis_tab<R, Dual<R>>(B, tab, kern, lev, Dual<R>(vx, nx), Dual<R>(vy, ny),
                                      Dual<R>(vz, nz), [&](int k, Dual<R> r) {
                                      const int sl = cnt & 15;
                                      W[sl][lane] = qv * r.v + dip * r.d;
                                      if (lane == 0) ks_slot[sl] = k;
                                      ++cnt;
                                      if ((cnt & 15) == 0) flush(16);
                                  });
        if (cnt & 15) flush(cnt & 15);
    }
    if (!multi) return;                                // uniform for the block
    __syncthreads();
    // a leaf of several chunks (it.cnt == 1): sum the waves' partials in
    // chunk order
    const int leaf = pm_leaf[it.first];
    if (T.level[leaf] < 2) return;
    const int nch = min(NCH, (it.tot + 63) / 64);
    for (int idx = threadIdx.x; idx < 2 * K; idx += blockDim.x) {
        const int kn = idx / K, k = idx - kn * K;
        R acc = part[kn * K + k];
        for (int c = 1; c < nch; ++c) acc += part[(c * 2 + kn) * K + k];
        M[((long long)leaf * 2 + kn) * K + k] = acc;
    }
}

// P2M by accumulation in registers (compile-time order PC): S adjacent lanes
// share one leaf and each sums the expansion of every S-th point of it (a
// fixed strided subset) in registers; the S partial expansions are then
// added across the lanes by a fixed butterfly.  The point loop has no LDS
// traffic and no barrier.  The orthonormalisation factors and, for the
// screened kernel, 1/g_n(kappa s) are constant over a leaf and are applied
// once to the sums.  Leaves come in order of decreasing point count, so the
// lanes of a wave run similar trip counts.  blockIdx.y is the kernel; with
// MS = 2, blockIdx.z picks one of two ranges of orders m (about half of the
// harmonics each), which halves the accumulators of a lane.
template <typename R, int PC, int S, int M0, int M1>
__device__ inline void p2m_acc_range(const BasisDev &B, const TreeDev &T,
                                     const BasisTab<R> &tab, const int *__restrict__ leaves,
                                     long long nleaf, const int *__restrict__ ptb,
                                     const int *__restrict__ pte, const R *px, const R *py,
                                     const R *pz, const R *pnx, const R *pny, const R *pnz,
                                     const R *sf, const R *sh, R inv_ebar, R *M) {
    constexpr int K = (PC + 1) * (PC + 1);
    constexpr int KS = solid_count(PC, M0, M1);
    const int kern = blockIdx.y;
    const long long slot = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / S;
    const int sub = threadIdx.x % S;
    const bool live = slot < nleaf;
    const int leaf = live ? leaves[slot] : 0;
    const int lev = live ? T.level[leaf] : 0;
    const int b = live ? ptb[leaf] : 0, e = live ? pte[leaf] : 0;
    const R cx = R(T.center[3 * leaf]), cy = R(T.center[3 * leaf + 1]);
    const R cz = R(T.center[3 * leaf + 2]);
    const R is = R(1.0 / B.side[lev]);
    const bool scr = kern == 1 && B.screened;         // uniform for the block
    const R ks = scr ? R(B.kappa * B.side[lev]) : R(0);
    R acc[KS];
#pragma unroll
    for (int j = 0; j < KS; ++j) acc[j] = R(0);
    for (int i = b + sub; i < e; i += S) {
        const Dual<R> ux((px[i] - cx) * is, pnx[i] * is), uy((py[i] - cy) * is, pny[i] * is);
        const Dual<R> uz((pz[i] - cz) * is, pnz[i] * is);
        const R qv = sh[i], dmag = -sf[i];
        const R dip = kern == 0 ? dmag * inv_ebar : dmag;
        int j = 0;                                    // static after unrolling
        if (!scr) {
            for_each_solid_p<PC, M0, M1, R>(ux, uy, uz, [&](int, int, Dual<R> r) {
                acc[j] += qv * r.v + dip * r.d;
                ++j;
            });
        } else {
            const Dual<R> t = (ks * ks) * ((ux * ux + uy * uy) + uz * uz);
            Dual<R> g[PC + 1];
            g_all_p<PC, R, Dual<R>>(t, tab.idf, tab.ser, g);
            for_each_solid_p<PC, M0, M1, R>(ux, uy, uz, [&](int, int n, Dual<R> r) {
                const Dual<R> w = r * g[n];
                acc[j] += qv * w.v + dip * w.d;
                ++j;
            });
        }
    }
#pragma unroll
    for (int j = 0; j < KS; ++j) {
#pragma unroll
        for (int o = 1; o < S; o <<= 1) acc[j] += __shfl_xor(acc[j], o, 64);
    }
    if (!live || sub != 0 || lev < 2) return;
    R *out = M + ((long long)leaf * 2 + kern) * K;
    const R *gi = tab.ginv + lev * (PC + 1);
    int j = 0;
    // the same (k, n) sequence; the harmonics themselves are dead code here
    for_each_solid_p<PC, M0, M1, R>(R(0), R(0), R(0), [&](int k, int n, R) {
        out[k] = acc[j] * (R(B.norm[k]) * (scr ? gi[n] : R(1)));
        ++j;
    });
}

template <typename R, int PC, int S, int MS>
__global__ void __launch_bounds__(256) k_p2m_acc(BasisDev B, TreeDev T,
                                                 const int *__restrict__ leaves, long long nleaf,
                                                 const int *__restrict__ ptb,
                                                 const int *__restrict__ pte,
                                                 const R *px, const R *py, const R *pz,
                                                 const R *pnx, const R *pny, const R *pnz,
                                                 const R *sf, const R *sh, R inv_ebar, R *M,
                                                 int nlev) {
    extern __shared__ __align__(16) unsigned char tab_raw[];
    const BasisTab<R> tab = stage_basis<R>(B, nlev, tab_raw);
    if constexpr (MS == 1) {
        p2m_acc_range<R, PC, S, 0, PC>(B, T, tab, leaves, nleaf, ptb, pte, px, py, pz, pnx, pny,
                                       pnz, sf, sh, inv_ebar, M);
    } else {
        constexpr int H = solid_split(PC);
        if (blockIdx.z == 0)
            p2m_acc_range<R, PC, S, 0, H - 1>(B, T, tab, leaves, nleaf, ptb, pte, px, py, pz,
                                              pnx, pny, pnz, sf, sh, inv_ebar, M);
        else
            p2m_acc_range<R, PC, S, H, PC>(B, T, tab, leaves, nleaf, ptb, pte, px, py, pz, pnx,
                                           pny, pnz, sf, sh, inv_ebar, M);
    }
}

// ---------------------------------------------------------------------------
// Batched K x K translations on the matrix cores.  One block (4 waves) owns a
// set of up to CC output columns; each wave owns a fixed subset of the
// 16 x 16 output tiles and runs v_mfma_*_16x16x4 over the (zero-padded) K
// dimension.  Operands: A = translation operator rows (read from cache),
// B = gathered expansions in LDS ([KK][CC]).
//   MODE 0  M2L, per-entry layout: one operator per work item (level,
//                offset class); column c = one V entry; result -> its
//                slot of Z (the grouped layout runs in k_m2l below)
//   MODE 1  M2M  eight operators (child octants) accumulated;
//                column c = one parent box; result -> M[parent]
//   MODE 2  L2L  eight operators, shared input L[parent];
//                result added to L[child of octant o]
// Operand layout of the 16x16x4 instructions (64 lanes, lane l, measured on
// gfx950):  A[i][k]: i = l % 16, k = l / 16;  B[k][j]: k = l / 16, j = l % 16;
//   D[i][j]: j = l % 16 and, for result register r = 0..3,
//            f32: i = 4 (l / 16) + r        f64: i = (l / 16) + 4 r.
// ---------------------------------------------------------------------------
struct TransArgs {
    int K, KK, nlev;
    int KZ;                      // M2L: slot length of one result (K rounded up to 16)
    long long nkey, PM;
    // M2L
    const int *item_ops, *item_begin, *item_count, *cols, *vgsrc;
    int vstride;                 // M2L: entries per group in vgsrc (8, or 1 per entry)
    // M2M / L2L
    long long lb, le;            // boxes of the parent level
    long long ncap;              // mode 1: capacity (boxes) of one octant slice of the scratch
    int n_items;                 // M2L: number of work items
    int nsplit;                  // M2L: blocks (and result slots) per group
    int KC;                      // bf16 M2L: 32-deep k-chunks
    long long PMB;               // bf16 M2L: elements per packed matrix (each part)
    const int *cb, *nc;          // child begin / count
    const unsigned long long *prefix;
    const int *pr_src, *pr_slot; // M2L pair layout: sources / result slots per octant
};

// Row stride (elements) of the gathered expansions in LDS, chosen so that
// the operand reads of one k-step (16 columns x 4 consecutive k) fall in
// distinct banks.
__host__ __device__ inline int lds_stride(int kk, int elem_bytes) {
    return elem_bytes == 4 ? kk + ((2 - kk) % 32 + 32) % 32 : (kk | 1);
}

// Result of one 16 x 16 output tile: destination offset of column col, or
// -1 when the column is absent.
template <typename R, int CC, int MODE>
__device__ inline long long trans_dst(const TransArgs &a, const int *colbox,
                                      const int (*child)[CC], int col, int o, int kern) {
    const int K = a.K;
    if (MODE == 0) {
        // slot of the group (target-major)
        (void)K;
        return ((long long)colbox[col] * 2 + kern) * a.KZ;
    } else if (MODE == 1) {
        // per-octant product of parent column col (summed by k_m2m_sum)
        return (((long long)o * a.ncap + (colbox[col] - a.lb)) * 2 + kern) * K;
    } else {
        const int ch = child[o][col];
        return ch < 0 ? -1 : ((long long)ch * 2 + kern) * K;
    }
}

template <typename R, int CC, int MODE, int NA>
__device__ inline void trans_store(const TransArgs &a, typename Acc4<R>::T (&acc)[NA],
                                   R *__restrict__ out, const int *colbox,
                                   const int (*child)[CC], int ncols, int o, int kern, int lane,
                                   int rt) {
#pragma unroll
    for (int ct = 0; ct < NA; ++ct) {
        const int col = ct * 16 + (lane & 15);
        if (col >= ncols) continue;
        const long long dst = trans_dst<R, CC, MODE>(a, colbox, child, col, o, kern);
        if (dst < 0) continue;
        if constexpr (MODE == 0 && sizeof(R) == sizeof(float)) {
            // M2L slots hold whole row tiles (KZ >= 16 NRT, 64-byte aligned):
            // the four consecutive rows of a lane go out as one 16-byte store
            *reinterpret_cast<typename Acc4<R>::T *>(out + dst + rt * 16 + 4 * (lane >> 4)) = acc[ct];
            continue;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int rr = rt * 16 + drow<R>(lane, r);
            if (MODE == 0 || rr < a.K) {     // M2L: rows past K are the slot's zero pad
                if (MODE == 2) out[dst + rr] += acc[ct][r];
                else out[dst + rr] = acc[ct][r];
            }
        }
    }
}

// Streaming form (any order): waves take row tiles in turn; operator
// fragments are loaded four k-steps ahead and each feeds NA products.
template <typename R, int CC, int MODE, int NA>
__device__ inline void trans_rows(const TransArgs &a, const R *__restrict__ op0, const R *Ms,
                                  int KKp, R *__restrict__ out, const int *colbox,
                                  const int (*child)[CC], int ncols, int o, int kern, int lane,
                                  int wave) {
    typedef typename Acc4<R>::T V4;
    const int K = a.K, KK = a.KK, KS = KK / 4;
    const int NRT = (K + 15) / 16;
    const R *Bp = Ms + (lane & 15) * KKp + (lane >> 4);
    const int nwave = (int)(blockDim.x >> 6);
    for (int rt = wave; rt < NRT; rt += nwave) {
        const R *A = op0 + (long long)rt * KS * 64 + lane;
        V4 acc[NA];
#pragma unroll
        for (int ct = 0; ct < NA; ++ct) acc[ct] = V4{0, 0, 0, 0};
        R pre[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) pre[j] = A[j * 64];
        for (int ks = 0; ks < KS; ks += 4) {
            R cur[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                cur[j] = pre[j];
                pre[j] = A[(ks + 4 + j) * 64];   // in bounds: operators carry a tail pad
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (ks + j < KS) {
#pragma unroll
                    for (int ct = 0; ct < NA; ++ct)
                        acc[ct] = mfma16(cur[j], Bp[ct * 16 * KKp + (ks + j) * 4], acc[ct]);
                }
            }
        }
        trans_store<R, CC, MODE, NA>(a, acc, out, colbox, child, ncols, o, kern, lane, rt);
    }
}

// Register-resident form (one row tile per wave, at most KSR k-steps): the
// wave's operator rows were loaded into areg before the operand gather; the
// product runs KSR k-steps from registers and LDS only (operand rows past K
// are zero in LDS, and so are the operator fragments past the operator's own
// k-steps: a non-finite value there would survive the multiplication by zero).
template <typename R, int CC, int MODE, int NA, int KSR>
__device__ inline void trans_rows_res(const TransArgs &a, const R (&areg)[KSR], const R *Ms,
                                      int KKp, R *__restrict__ out, const int *colbox,
                                      const int (*child)[CC], int ncols, int o, int kern,
                                      int lane, int rt) {
    typedef typename Acc4<R>::T V4;
    const R *Bp = Ms + (lane & 15) * KKp + (lane >> 4);
    V4 acc[NA];
#pragma unroll
    for (int ct = 0; ct < NA; ++ct) acc[ct] = V4{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < KSR; ++ks) {
#pragma unroll
        for (int ct = 0; ct < NA; ++ct)
            acc[ct] = mfma16(areg[ks], Bp[ct * 16 * KKp + ks * 4], acc[ct]);
    }
    trans_store<R, CC, MODE, NA>(a, acc, out, colbox, child, ncols, o, kern, lane, rt);
}

// Gathers the B operand of one block: column c (c < 16 nact) of Ms holds
// rows [0, KR) of the expansion of box srcbox[c] (zero past K and for
// absent columns).
template <typename R>
__device__ inline void gather_cols(const R *__restrict__ in, const int *srcbox, int ncols,
                                   int nact, int K, int KR, int KKp, int kern, int lane,
                                   int wave, R *Ms) {
    // gather the B operand column by column (consecutive lanes read
    // consecutive coefficients of one expansion); a wave issues the loads of
    // four columns before it stores any, so their latencies overlap.  Rows
    // past K and missing columns are zero.
    {
        const int nwave = (int)(blockDim.x >> 6);
        const int ncs = nact * 16;
        for (int c0 = wave; c0 < ncs; c0 += 4 * nwave) {
            R v[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int c = c0 + u * nwave;
                const int src = (c < ncols) ? srcbox[c] : -1;
                const R *col = in + ((long long)(src < 0 ? 0 : src) * 2 + kern) * K;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int k = lane + 64 * j;
                    v[u][j] = (src >= 0 && k < K) ? col[k] : R(0);
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int c = c0 + u * nwave;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int k = lane + 64 * j;
                    if (c < ncs && k < KR) Ms[c * KKp + k] = v[u][j];
                }
            }
            // rows past 256 (expansion order above 14)
            for (int u = 0; u < 4; ++u) {
                const int c = c0 + u * nwave;
                if (c >= ncs) break;
                const int src = (c < ncols) ? srcbox[c] : -1;
                const R *col = in + ((long long)(src < 0 ? 0 : src) * 2 + kern) * K;
                for (int k = lane + 256; k < KR; k += 64)
                    Ms[c * KKp + k] = (src >= 0 && k < K) ? col[k] : R(0);
            }
        }
    }
}

template <typename R, int CC, int MODE, int KSR>
__global__ void __launch_bounds__(512) k_trans(TransArgs a, const R *__restrict__ ops,
                                               const R *__restrict__ in, R *__restrict__ out,
                                               int lev) {
    extern __shared__ unsigned char smem_raw[];
    R *Ms = reinterpret_cast<R *>(smem_raw);         // [CC][KKp]
    __shared__ int colbox[CC];                         // mode 0: V entry; 1, 2: parent box
    __shared__ int srcbox[CC];                         // box whose expansion is column c
    __shared__ int child[8][CC];                       // modes 1, 2: child of octant o
    const int K = a.K, KK = a.KK, KS = KK / 4;
    // operand rows held in LDS: KK, or all KSR k-steps of the resident form
    const int KR = KSR > 0 ? 4 * KSR : KK;
    const int KKp = lds_stride(KR, (int)sizeof(R));
    const int kern = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int o = (MODE == 0) ? 0 : (int)blockIdx.z;  // child octant (modes 1, 2)
    int ncols;
    const R *op0;
    if (MODE == 0) {
        // Work item w, columns [blockIdx.z * CC, +CC) of its <= 64 entries.
        // Blocks are dealt to the 8 XCDs in turn (block b runs on XCD b % 8);
        // XCD x takes the contiguous item range [x per, (x+1) per), so the
        // items of one (level, class) bucket share their operator in one L2.
        // gridDim.x = 8 per, so b -> w is a bijection onto [0, 8 per).
        const int per = (int)(gridDim.x >> 3);
        const int w = (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
        if (w >= a.n_items) return;                      // uniform for the block
        const int off = blockIdx.z * CC;
        ncols = min(CC, a.item_count[w] - off);
        if (ncols <= 0) return;                          // uniform for the block
        const int beg = a.item_begin[w] + off;
        if (tid < CC) {
            const int q = tid < ncols ? a.cols[beg + tid] : -1;
            colbox[tid] = q;
            srcbox[tid] = q >= 0 ? a.vgsrc[q] : -1;
        }
        op0 = ops + ((long long)kern * a.nkey + a.item_ops[8 * (long long)w]) * a.PM;
    } else {
        const long long c0 = a.lb + (long long)blockIdx.x * CC;
        ncols = (int)min((long long)CC, a.le - c0);
        if (tid < CC) {
            colbox[tid] = tid < ncols ? (int)(c0 + tid) : -1;
            for (int q = 0; q < 8; ++q) child[q][tid] = -1;
            if (tid < ncols) {
                const int P = (int)(c0 + tid);
                for (int c = a.cb[P]; c < a.cb[P] + a.nc[P]; ++c)
                    child[(int)(a.prefix[c] & 7ull)][tid] = c;
            }
        }
        op0 = ops + ((((long long)kern * a.nlev + lev) * 8) + o) * a.PM;
    }
    // resident form: this wave's operator rows (row tile = wave), issued now
    // so that their latency overlaps the operand gather
    R areg[KSR > 0 ? KSR : 1];
    if constexpr (KSR > 0) {
        const R *A = op0 + (long long)wave * KS * 64 + lane;
#pragma unroll
        // k-steps past the operator's KS are zero in registers: the values
        // beyond belong to the next matrix (or are unwritten), and although
        // the matching operand rows in LDS are zero, NaN * 0 would be NaN
        for (int j = 0; j < KSR; ++j) areg[j] = j < KS ? A[j * 64] : R(0);
    }
    __syncthreads();
    if (MODE != 0 && tid < CC) srcbox[tid] = (MODE == 1) ? child[o][tid] : colbox[tid];
    __syncthreads();
    const int nact = (ncols + 15) / 16;                  // active column tiles
    gather_cols<R>(in, srcbox, ncols, nact, K, KR, KKp, kern, lane, wave, Ms);
    __syncthreads();
    if constexpr (KSR > 0) {
        if constexpr (CC >= 64) {
            if (nact == 4) { trans_rows_res<R, CC, MODE, 4, KSR>(a, areg, Ms, KKp, out, colbox, child, ncols, o, kern, lane, wave); return; }
            if (nact == 3) { trans_rows_res<R, CC, MODE, 3, KSR>(a, areg, Ms, KKp, out, colbox, child, ncols, o, kern, lane, wave); return; }
        }
        if constexpr (CC >= 32) {
            if (nact == 2) { trans_rows_res<R, CC, MODE, 2, KSR>(a, areg, Ms, KKp, out, colbox, child, ncols, o, kern, lane, wave); return; }
        }
        trans_rows_res<R, CC, MODE, 1, KSR>(a, areg, Ms, KKp, out, colbox, child, ncols, o, kern, lane, wave);
    } else {
        if constexpr (CC >= 64) {
            if (nact == 4) { trans_rows<R, CC, MODE, 4>(a, op0, Ms, KKp, out, colbox, child, ncols, o, kern, lane, wave); return; }
            if (nact == 3) { trans_rows<R, CC, MODE, 3>(a, op0, Ms, KKp, out, colbox, child, ncols, o, kern, lane, wave); return; }
        }
        if constexpr (CC >= 32) {
            if (nact == 2) { trans_rows<R, CC, MODE, 2>(a, op0, Ms, KKp, out, colbox, child, ncols, o, kern, lane, wave); return; }
        }
        trans_rows<R, CC, MODE, 1>(a, op0, Ms, KKp, out, colbox, child, ncols, o, kern, lane, wave);
    }
}

// ---------------------------------------------------------------------------
// M2L by groups (k_m2l; the bf16 M2L below takes both layouts).  A work item
// is <= 64 groups of one bucket; every group of the bucket takes the same
// operator in octant slot c.  Grouped layout: a group is the V entries of
// one target that are children of one colleague of its parent (bucket:
// level, colleague offset, target octant).  Per-entry layout: a group is one
// V entry (bucket: level, offset class; one octant slot).  For each octant
// slot with an operator the block gathers that child's expansions of its
// columns into LDS and each wave adds its operator row tile times them to
// its accumulators, so the sum over a group's children leaves the registers
// once, into the group's slot of Z.  Operator fragments stream from cache
// four k-steps ahead.
// ---------------------------------------------------------------------------
// Share h of nsplit of an item's octants with operators: ranks [lo, hi)
// among them, in octant order (an empty share stores zeros).
__device__ inline void m2l_share(const int *__restrict__ iops, int nsplit, int h, int &lo,
                                 int &hi) {
    int n = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) n += iops[c] >= 0;
    const int per = (n + nsplit - 1) / nsplit;
    lo = min(n, h * per);
    hi = min(n, lo + per);
}

template <typename R, int CC, int NA>
__device__ inline void m2l_group_rows(const TransArgs &a, const R *__restrict__ ops,
                                      const R *__restrict__ in, R *__restrict__ out, R *Ms,
                                      int KKp, const int *colbox, const int (*srcbox)[CC],
                                      const int *__restrict__ iops, int lo, int hi, int ncols,
                                      int kern, int lane, int wave) {
    typedef typename Acc4<R>::T V4;
    const int K = a.K, KK = a.KK, KS = KK / 4, NRT = (K + 15) / 16;
    const int nwave = (int)(blockDim.x >> 6);
    const R *Bp = Ms + (lane & 15) * KKp + (lane >> 4);
    for (int rt0 = 0; rt0 < NRT; rt0 += nwave) {
        const int rt = rt0 + wave;
        if (rt0 > 0) __syncthreads();                    // the last pass's products done
        V4 acc[NA];
#pragma unroll
        for (int ct = 0; ct < NA; ++ct) acc[ct] = V4{0, 0, 0, 0};
        bool busy = false;                               // an octant was multiplied
        for (int c = 0, rank = 0; c < 8; ++c) {
            const int key = __builtin_amdgcn_readfirstlane(iops[c]);   // uniform
            if (key < 0 || rank++ < lo || rank > hi) continue;         // not this block's
            if (busy) __syncthreads();                   // products of the last octant done
            busy = true;
            gather_cols<R>(in, srcbox[c], ncols, NA, K, KK, KKp, kern, lane, wave, Ms);
            __syncthreads();
            if (rt >= NRT) continue;
            const R *A = ops + ((long long)kern * a.nkey + key) * a.PM +
                         (long long)rt * KS * 64 + lane;
            R pre[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) pre[j] = A[j * 64];
            for (int ks = 0; ks < KS; ks += 4) {
                R cur[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    cur[j] = pre[j];
                    pre[j] = A[(ks + 4 + j) * 64];       // in bounds: operators carry a tail pad
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (ks + j < KS) {
#pragma unroll
                        for (int ct = 0; ct < NA; ++ct)
                            acc[ct] = mfma16(cur[j], Bp[ct * 16 * KKp + (ks + j) * 4], acc[ct]);
                    }
                }
            }
        }
        if (rt < NRT)
            trans_store<R, CC, 0, NA>(a, acc, out, colbox, nullptr, ncols, 0, kern, lane, rt);
    }
}

template <typename R, int CC>
__global__ void __launch_bounds__(1024)
__attribute__((amdgpu_waves_per_eu(sizeof(R) == sizeof(float) ? 8 : 1)))
k_m2l(TransArgs a, const R *__restrict__ ops,
                                              const R *__restrict__ in, R *__restrict__ out) {
    extern __shared__ unsigned char smem_raw[];
    R *Ms = reinterpret_cast<R *>(smem_raw);          // [CC][KKp]
    __shared__ int colbox[CC];                         // group of column c
    __shared__ int srcbox[8][CC];                      // its child in octant o (or -1)
    const int KKp = lds_stride(a.KK, (int)sizeof(R));
    const int kern = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // Work item w, columns [blockIdx.z * CC, +CC) of its <= 64 groups.
    // Blocks are dealt to the 8 XCDs in turn (block b runs on XCD b % 8);
    // XCD x takes the contiguous item range [x per, (x+1) per), so items of
    // one bucket, which share their operators, share one L2.
    // gridDim.x = 8 per, so b -> w is a bijection onto [0, 8 per).
    const int per = (int)(gridDim.x >> 3);
    const int w = (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
    if (w >= a.n_items) return;                        // uniform for the block
    // blockIdx.z = column chunk * nsplit + part: part h takes the h-th share
    // of the item's octants (in octant order) and writes slot h of each group
    const int h = (int)blockIdx.z % a.nsplit;
    const int off = ((int)blockIdx.z / a.nsplit) * CC;
    const int ncols = min(CC, a.item_count[w] - off);
    if (ncols <= 0) return;                            // uniform for the block
    const int beg = a.item_begin[w] + off;
    const int *iops = a.item_ops + 8 * (long long)w;
    int lo, hi;
    m2l_share(iops, a.nsplit, h, lo, hi);
    if (tid < CC) {
        const int g = tid < ncols ? a.cols[beg + tid] : -1;
        colbox[tid] = g >= 0 ? g * a.nsplit + h : -1;
#pragma unroll
        for (int o = 0; o < 8; ++o)
            srcbox[o][tid] = (g >= 0 && iops[o] >= 0) ? a.vgsrc[(long long)g * a.vstride + o] : -1;
    }
    __syncthreads();               // column tables visible to every wave
    const int nact = (ncols + 15) / 16;                // active column tiles
    if constexpr (CC >= 64) {
        if (nact == 4) { m2l_group_rows<R, CC, 4>(a, ops, in, out, Ms, KKp, colbox, srcbox, iops, lo, hi, ncols, kern, lane, wave); return; }
        if (nact == 3) { m2l_group_rows<R, CC, 3>(a, ops, in, out, Ms, KKp, colbox, srcbox, iops, lo, hi, ncols, kern, lane, wave); return; }
    }
    if constexpr (CC >= 32) {
        if (nact == 2) { m2l_group_rows<R, CC, 2>(a, ops, in, out, Ms, KKp, colbox, srcbox, iops, lo, hi, ncols, kern, lane, wave); return; }
    }
    m2l_group_rows<R, CC, 1>(a, ops, in, out, Ms, KKp, colbox, srcbox, iops, lo, hi, ncols, kern, lane, wave);
}

// M2L by pairs of boxes (k_m2l_pairs).  A work item is <= CC pairs (P, C)
// of one level and one colleague offset; for each source octant c the block
// gathers child c of every pair's C into LDS once, and the waves multiply it
// by the operators of all eight target octants, accumulating per (target
// octant, row tile) in registers (JPW such jobs per wave).  At the end each
// job's tile goes to the slot of (child b of P, C) of the grouped layout, so
// that the grouped reduction over colleagues applies unchanged.  Against the
// grouped layout, each source expansion is read once per pair instead of
// once per child of P.
template <typename R, int CC, int NA, int JPW>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4)))
k_m2l_pairs(TransArgs a, const R *__restrict__ ops, const R *__restrict__ in,
            R *__restrict__ out) {
    typedef typename Acc4<R>::T V4;
    extern __shared__ unsigned char smem_raw[];
    R *Ms = reinterpret_cast<R *>(smem_raw);          // [CC][KKp]
    __shared__ int src[8][CC], slot[8][CC], iops[64];
    const int KKp = lds_stride(a.KK, (int)sizeof(R));
    const int kern = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nwave = (int)(blockDim.x >> 6);
    // items dealt to the XCDs in contiguous ranges (block b runs on XCD b % 8)
    const int per = (int)(gridDim.x >> 3);
    const int w = (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
    if (w >= a.n_items) return;                        // uniform for the block
    // columns [blockIdx.z CC, + CC) of the item's <= 64 pairs
    const int off = (int)blockIdx.z * CC;
    const int ncols = min(CC, a.item_count[w] - off);
    if (ncols <= 0) return;                            // uniform for the block
    const int beg = a.item_begin[w] + off;
    for (int i = tid; i < 8 * CC; i += blockDim.x) {
        const int o = i / CC, col = i % CC;
        const bool ok = col < ncols;
        src[o][col] = ok ? a.pr_src[8 * (long long)(beg + col) + o] : -1;
        slot[o][col] = ok ? a.pr_slot[8 * (long long)(beg + col) + o] : -1;
    }
    if (tid < 64) iops[tid] = a.item_ops[64 * (long long)w + tid];
    __syncthreads();
    const int K = a.K, KK = a.KK, KS = KK / 4, NRT = (K + 15) / 16;
    // K = 16 (NRT - 1) + 1 (orders 6, 8, 14): the last row tile would hold one
    // row, so that row is a dot product on the vector ALU instead (one
    // column per lane, waves 8..15 for target octants 0..7), and the matrix
    // cores take NRT - 1 row tiles
    const bool tail = K == 16 * (NRT - 1) + 1;
    const int MRT = tail ? NRT - 1 : NRT;
    const R *Bp = Ms + (lane & 15) * KKp + (lane >> 4);
    V4 acc[JPW][NA];
#pragma unroll
    for (int q = 0; q < JPW; ++q)
#pragma unroll
        for (int ct = 0; ct < NA; ++ct) acc[q][ct] = V4{0, 0, 0, 0};
    R tacc = R(0);                                     // tail row, column `lane`
    const int tb = wave - 8;                           // tail target octant of this wave
    bool busy = false;
    for (int c = 0; c < 8; ++c) {
        int any = 0;
#pragma unroll
        for (int b = 0; b < 8; ++b) any |= iops[8 * b + c] >= 0;
        if (!__builtin_amdgcn_readfirstlane(any)) continue;   // uniform
        if (busy) __syncthreads();                     // products of the last octant done
        busy = true;
        gather_cols<R>(in, src[c], ncols, NA, K, KK, KKp, kern, lane, wave, Ms);
        __syncthreads();
        if (tail && tb >= 0) {                         // uniform for the wave
            const int key = __builtin_amdgcn_readfirstlane(iops[8 * tb + c]);
            if (key >= 0 && lane < ncols) {
                // row K - 1 of the operator: fragment (MRT, k / 4), lane 16 (k % 4)
                const R *A = ops + ((long long)kern * a.nkey + key) * a.PM +
                             (long long)MRT * KS * 64;
                const R *m = Ms + lane * KKp;
                for (int k = 0; k < K; ++k) tacc += A[(k >> 2) * 64 + (k & 3) * 16] * m[k];
            }
        }
#pragma unroll
        for (int q = 0; q < JPW; ++q) {
            const int j = wave + q * nwave;
            if (j >= 8 * MRT) continue;               // uniform for the wave
            const int b = j / MRT, rt = j - b * MRT;
            const int key = __builtin_amdgcn_readfirstlane(iops[8 * b + c]);
            if (key < 0) continue;
            const R *A = ops + ((long long)kern * a.nkey + key) * a.PM +
                         (long long)rt * KS * 64 + lane;
            R pre[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) pre[u] = A[u * 64];
            for (int ks = 0; ks < KS; ks += 4) {
                R cur[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    cur[u] = pre[u];
                    pre[u] = A[(ks + 4 + u) * 64];     // in bounds: operators carry a tail pad
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (ks + u < KS) {
#pragma unroll
                        for (int ct = 0; ct < NA; ++ct)
                            acc[q][ct] = mfma16(cur[u], Bp[ct * 16 * KKp + (ks + u) * 4], acc[q][ct]);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < JPW; ++q) {
        const int j = wave + q * nwave;
        if (j >= 8 * MRT) continue;
        const int b = j / MRT, rt = j - b * MRT;
        trans_store<R, CC, 0, NA>(a, acc[q], out, slot[b], nullptr, ncols, 0, kern, lane, rt);
    }
    if (tail && tb >= 0 && lane < ncols && slot[tb][lane] >= 0)
        out[((long long)slot[tb][lane] * 2 + kern) * a.KZ + K - 1] = tacc;
}

// ---------------------------------------------------------------------------
// M2L with bf16-split operands on the 16x16x32 bf16 matrix instruction: each
// FP32 value v = hi + lo with hi = bf16(v), lo = bf16(v - hi); the product
// T m is taken as hi(T) hi(m) + hi(T) lo(m) + lo(T) hi(m) (the lo*lo term,
// about 2^-16 of the product, is dropped), accumulated in FP32.  Operand
// layout (measured on gfx950): lane l, element e holds A[l%16][8 (l/16) + e]
// and B[8 (l/16) + e][l%16] of each 32-deep chunk; results as the FP32
// 16x16x4 instruction.  Same work items, XCD mapping and outputs as the
// FP32 M2L.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8_t __attribute__((ext_vector_type(8)));

__device__ inline unsigned short bf16_bits(float v) {
    return __builtin_bit_cast(unsigned short, (__bf16)v);
}
__device__ inline float bf16_value(unsigned short b) {
    return (float)__builtin_bit_cast(__bf16, b);
}
__device__ inline f4v mfma_bf16(u16x8_t a, u16x8_t b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                   __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
}

// Row stride (elements) of the bf16 operand rows in LDS: a multiple of 8 (16 B
// reads) with an odd number of 16-byte units, so that 16 columns read at one
// k offset hit 16 different 16-byte bank groups.
__host__ __device__ inline int bf16_stride(int kr) {
    int u = (kr + 7) / 8;
    if ((u & 1) == 0) ++u;
    return 8 * u;
}

template <int CC, int NA, bool GROUPED>
__device__ inline void m2l_bf16_group(const TransArgs &a, const u16x8_t *__restrict__ opsh,
                                      const u16x8_t *__restrict__ opsl,
                                      const float *__restrict__ in, float *__restrict__ out,
                                      unsigned short *Mh, unsigned short *Ml, int KKp,
                                      const int *colbox, const int (*srcbox)[CC],
                                      const int *__restrict__ iops, int lo, int hi, int ncols,
                                      int kern, int lane, int wave) {
    const int K = a.K, KC = a.KC, KR = 32 * KC, NRT = (K + 15) / 16;
    const int nwave = (int)(blockDim.x >> 6);
    const int boff = (lane & 15) * KKp + 8 * (lane >> 4);
    for (int rt0 = 0; rt0 < NRT; rt0 += nwave) {
        const int rt = rt0 + wave;
        if (rt0 > 0) __syncthreads();                    // the last pass's products done
        f4v acc[NA];
#pragma unroll
        for (int ct = 0; ct < NA; ++ct) acc[ct] = f4v{0, 0, 0, 0};
        bool busy = false;                               // an octant was multiplied
        for (int c = 0, rank = 0; c < (GROUPED ? 8 : 1); ++c) {
            const int key = __builtin_amdgcn_readfirstlane(iops[c]);
            if (key < 0 || rank++ < lo || rank > hi) continue;         // not this block's
            if (busy) __syncthreads();                   // products of the last octant done
            busy = true;
            for (int col = wave; col < NA * 16; col += nwave) {
                const int src = col < ncols ? srcbox[c][col] : -1;
                const float *cp = in + ((long long)(src < 0 ? 0 : src) * 2 + kern) * K;
                for (int k = lane; k < KR; k += 64) {
                    const float v = (src >= 0 && k < K) ? cp[k] : 0.0f;
                    const unsigned short h = bf16_bits(v);
                    Mh[col * KKp + k] = h;
                    Ml[col * KKp + k] = bf16_bits(v - bf16_value(h));
                }
            }
            __syncthreads();
            if (rt >= NRT) continue;
            const long long mat = (long long)kern * a.nkey + key;
            const u16x8_t *Ah = opsh + mat * (a.PMB / 8) + (long long)rt * KC * 64 + lane;
            const u16x8_t *Al = opsl + mat * (a.PMB / 8) + (long long)rt * KC * 64 + lane;
            u16x8_t ph = Ah[0], pl = Al[0];
            for (int kc = 0; kc < KC; ++kc) {
                const u16x8_t ah = ph, al = pl;
                ph = Ah[(kc + 1) * 64];        // in bounds: operators carry a tail pad
                pl = Al[(kc + 1) * 64];
#pragma unroll
                for (int ct = 0; ct < NA; ++ct) {
                    const int o = ct * 16 * KKp + boff + 32 * kc;
                    const u16x8_t bh = *reinterpret_cast<const u16x8_t *>(Mh + o);
                    const u16x8_t bl = *reinterpret_cast<const u16x8_t *>(Ml + o);
                    acc[ct] = mfma_bf16(ah, bh, acc[ct]);
                    acc[ct] = mfma_bf16(ah, bl, acc[ct]);
                    acc[ct] = mfma_bf16(al, bh, acc[ct]);
                }
            }
        }
        if (rt >= NRT) continue;
#pragma unroll
        for (int ct = 0; ct < NA; ++ct) {
            const int col = ct * 16 + (lane & 15);
            if (col >= ncols) continue;
            const long long dst = ((long long)colbox[col] * 2 + kern) * a.KZ;
            *reinterpret_cast<f4v *>(out + dst + rt * 16 + 4 * (lane >> 4)) = acc[ct];
        }
    }
}

// One block per work item (as the FP32 M2L: groups, XCD-contiguous items);
// waves take the operators' row tiles, fragments loaded one chunk ahead.
template <int CC, bool GROUPED>
__global__ void __launch_bounds__(1024) k_m2l_bf16(TransArgs a, const u16x8_t *__restrict__ opsh,
                                                   const u16x8_t *__restrict__ opsl,
                                                   const float *__restrict__ in,
                                                   float *__restrict__ out) {
    extern __shared__ __align__(16) unsigned char smem_bf[];
    __shared__ int colbox[CC];
    __shared__ int srcbox[8][CC];
    const int KR = 32 * a.KC, KKp = bf16_stride(KR);
    unsigned short *Mh = reinterpret_cast<unsigned short *>(smem_bf);    // [CC][KKp]
    unsigned short *Ml = Mh + CC * KKp;
    const int kern = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int per = (int)(gridDim.x >> 3);
    const int w = (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
    if (w >= a.n_items) return;
    // blockIdx.z = column chunk * nsplit + part: part h takes the h-th share
    // of the item's octants (in octant order) and writes slot h of each group
    const int h = (int)blockIdx.z % a.nsplit;
    const int off = ((int)blockIdx.z / a.nsplit) * CC;
    const int ncols = min(CC, a.item_count[w] - off);
    if (ncols <= 0) return;                            // uniform for the block
    const int beg = a.item_begin[w] + off;
    const int *iops = a.item_ops + 8 * (long long)w;
    int lo, hi;
    m2l_share(iops, a.nsplit, h, lo, hi);
    if (tid < CC) {
        const int g = tid < ncols ? a.cols[beg + tid] : -1;
        colbox[tid] = g >= 0 ? g * a.nsplit + h : -1;
#pragma unroll
        for (int o = 0; o < (GROUPED ? 8 : 1); ++o)
            srcbox[o][tid] = (g >= 0 && iops[o] >= 0) ? a.vgsrc[(long long)g * a.vstride + o] : -1;
    }
    __syncthreads();               // column tables visible to every wave
    const int nact = (ncols + 15) / 16;
    if constexpr (CC >= 64) {
        if (nact == 4) { m2l_bf16_group<CC, 4, GROUPED>(a, opsh, opsl, in, out, Mh, Ml, KKp, colbox, srcbox, iops, lo, hi, ncols, kern, lane, wave); return; }
        if (nact == 3) { m2l_bf16_group<CC, 3, GROUPED>(a, opsh, opsl, in, out, Mh, Ml, KKp, colbox, srcbox, iops, lo, hi, ncols, kern, lane, wave); return; }
    }
    if constexpr (CC >= 32) {
        if (nact == 2) { m2l_bf16_group<CC, 2, GROUPED>(a, opsh, opsl, in, out, Mh, Ml, KKp, colbox, srcbox, iops, lo, hi, ncols, kern, lane, wave); return; }
    }
    m2l_bf16_group<CC, 1, GROUPED>(a, opsh, opsl, in, out, Mh, Ml, KKp, colbox, srcbox, iops, lo, hi, ncols, kern, lane, wave);
}

// threads per M2L block: one wave per operator row tile, at most 16 (larger
// orders take the row tiles in balanced passes)
inline unsigned m2l_threads(int K) {
    const int nrt = (K + 15) / 16, passes = (nrt + 15) / 16;
    return 64u * (unsigned)((nrt + passes - 1) / passes);
}

void launch_m2l_bf16(const TransArgs &ta, unsigned gx, bool grouped, const u16x8_t *opsh,
                     const u16x8_t *opsl, const float *in, float *out, hipStream_t s) {
    const unsigned nthr = m2l_threads(ta.K), ns = (unsigned)ta.nsplit;
    (void)blocks_ok(gx, nthr);
    const size_t kkp = (size_t)bf16_stride(32 * ta.KC);
    auto shmem = [&](int cc) { return 2 * kkp * cc * sizeof(unsigned short); };
    const size_t lim = 60 * 1024;
    if (shmem(64) <= lim) {
        if (grouped) k_m2l_bf16<64, true><<<dim3(gx, 2, 1 * ns), nthr, shmem(64), s>>>(ta, opsh, opsl, in, out);
        else k_m2l_bf16<64, false><<<dim3(gx, 2, 1 * ns), nthr, shmem(64), s>>>(ta, opsh, opsl, in, out);
    } else if (shmem(32) <= lim) {
        if (grouped) k_m2l_bf16<32, true><<<dim3(gx, 2, 2 * ns), nthr, shmem(32), s>>>(ta, opsh, opsl, in, out);
        else k_m2l_bf16<32, false><<<dim3(gx, 2, 2 * ns), nthr, shmem(32), s>>>(ta, opsh, opsl, in, out);
    } else {
        require(shmem(16) <= lim, ST_INVALID, "expansion order too large for the bf16 M2L");
        if (grouped) k_m2l_bf16<16, true><<<dim3(gx, 2, 4 * ns), nthr, shmem(16), s>>>(ta, opsh, opsl, in, out);
        else k_m2l_bf16<16, false><<<dim3(gx, 2, 4 * ns), nthr, shmem(16), s>>>(ta, opsh, opsl, in, out);
    }
    KCHK();
}

// Grouped FP32 / FP64 M2L (k_m2l): the widest column block that fits the
// LDS budget
template <typename R>
void launch_m2l(const TransArgs &ta, unsigned gx, const R *ops, const R *in, R *out,
                hipStream_t s) {
    const unsigned nthr = m2l_threads(ta.K), ns = (unsigned)ta.nsplit;
    (void)blocks_ok(gx, nthr);
    const size_t lim = 60 * 1024;
    auto shmem = [&](int cc) { return (size_t)lds_stride(ta.KK, (int)sizeof(R)) * cc * sizeof(R); };
    if (shmem(64) <= lim) {
        k_m2l<R, 64><<<dim3(gx, 2, 1 * ns), nthr, shmem(64), s>>>(ta, ops, in, out);
    } else if (shmem(32) <= lim) {
        k_m2l<R, 32><<<dim3(gx, 2, 2 * ns), nthr, shmem(32), s>>>(ta, ops, in, out);
    } else {
        require(shmem(16) <= lim, ST_INVALID, "expansion order too large for the translation kernels");
        k_m2l<R, 16><<<dim3(gx, 2, 4 * ns), nthr, shmem(16), s>>>(ta, ops, in, out);
    }
    KCHK();
}

// M2L in the pair layout: 16 waves, JPW = (8 row-tile count) / 16 jobs per
// wave; 64 columns up to order 10, above that two blocks of 32 columns per
// item (accumulator registers).
// Returns false where the grouped kernel runs instead (orders without an
// instantiation; FP64 above order 6).
template <typename R>
bool launch_m2l_pairs(const TransArgs &ta, unsigned gx, const R *ops, const R *in, R *out,
                      hipStream_t s) {
    const int nrt = (ta.K + 15) / 16;
    const int mrt = ta.K == 16 * (nrt - 1) + 1 ? nrt - 1 : nrt;   // row tiles on the matrix cores
    const int jpw = (8 * mrt + 15) / 16;
    // FP64 accumulators of more than two jobs spill at 128 VGPRs
    if (sizeof(R) == sizeof(double) && jpw > 2) return false;
    (void)blocks_ok(gx, 1024);
    auto shmem = [&](int cc) { return (size_t)lds_stride(ta.KK, (int)sizeof(R)) * cc * sizeof(R); };
    switch (jpw) {
        case 2: k_m2l_pairs<R, 64, 4, 2><<<dim3(gx, 2), 1024, shmem(64), s>>>(ta, ops, in, out); break;
        case 3:
            if constexpr (sizeof(R) == sizeof(float))
                k_m2l_pairs<R, 64, 4, 3><<<dim3(gx, 2), 1024, shmem(64), s>>>(ta, ops, in, out);
            break;
        case 4:
            if constexpr (sizeof(R) == sizeof(float))
                k_m2l_pairs<R, 64, 4, 4><<<dim3(gx, 2), 1024, shmem(64), s>>>(ta, ops, in, out);
            break;
        case 7:
        case 8:
            if constexpr (sizeof(R) == sizeof(float))
                k_m2l_pairs<R, 32, 2, 8><<<dim3(gx, 2, 2), 1024, shmem(32), s>>>(ta, ops, in, out);
            break;
        default: return false;
    }
    KCHK();
    return true;
}

// packed bf16 parts of the M2L operators (from the FP64 operators)
__global__ void k_pack_bf16(const double *__restrict__ src, long long nmat, int K, int KC,
                            int NRT, unsigned short *__restrict__ hi,
                            unsigned short *__restrict__ lo) {
    const long long PMB = (long long)NRT * KC * 64 * 8;
    long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nmat * PMB) return;
    const long long m = id / PMB;
    long long r = id % PMB;
    const int e = (int)(r % 8);
    r /= 8;
    const int l = (int)(r % 64);
    r /= 64;
    const int kc = (int)(r % KC), rt = (int)(r / KC);
    const int row = rt * 16 + (l & 15), k = kc * 32 + 8 * (l >> 4) + e;
    const double v = (row < K && k < K) ? src[m * K * K + (long long)row * K + k] : 0.0;
    const unsigned short h = bf16_bits((float)v);
    hi[id] = h;
    lo[id] = bf16_bits((float)(v - (double)bf16_value(h)));
}

// M of the non-leaf boxes of one level = sum over the 8 octant products.
template <typename R>
__global__ void k_m2m_sum(int K, long long lb, long long le, long long ncap,
                          const int *__restrict__ nc, const R *__restrict__ part,
                          R *__restrict__ M) {
    const long long P = lb + blockIdx.x;
    if (P >= le || nc[P] == 0) return;
    for (int idx = threadIdx.x; idx < 2 * K; idx += blockDim.x) {
        R acc = R(0);
#pragma unroll
        for (int q = 0; q < 8; ++q) acc += part[((long long)q * ncap + (P - lb)) * 2 * K + idx];
        M[P * 2 * K + idx] = acc;
    }
}

template <typename R, int MODE, int KSR>
void launch_trans_k(const TransArgs &ta, dim3 g, unsigned nthr, const R *ops, const R *in,
                    R *out, int lev, hipStream_t s) {
    const size_t lim = 60 * 1024;
    (void)blocks_ok(g.x, nthr);   // per grid dimension
    const int KR = KSR > 0 ? 4 * KSR : ta.KK;
    auto shmem = [&](int cc) { return (size_t)lds_stride(KR, (int)sizeof(R)) * cc * sizeof(R); };
    if (MODE == 0) {
        if (shmem(64) <= lim) {
            g.z = 1;
            k_trans<R, 64, 0, KSR><<<g, nthr, shmem(64), s>>>(ta, ops, in, out, lev);
        } else if (shmem(32) <= lim) {
            g.z = 2;
            k_trans<R, 32, 0, KSR><<<g, nthr, shmem(32), s>>>(ta, ops, in, out, lev);
        } else if (shmem(16) <= lim) {
            g.z = 4;
            k_trans<R, 16, 0, KSR><<<g, nthr, shmem(16), s>>>(ta, ops, in, out, lev);
        } else {
            throw Error(ST_INVALID, "expansion order too large for the translation kernels");
        }
    } else {
        require(shmem(16) <= lim, ST_INVALID, "expansion order too large for the translation kernels");
        g = dim3((unsigned)((ta.le - ta.lb + 15) / 16), 2, 8);
        k_trans<R, 16, MODE, KSR><<<g, nthr, shmem(16), s>>>(ta, ops, in, out, lev);
    }
    KCHK();
}

// M2M / L2L with up to 8 row tiles and 32 k-steps (p <= 10): one wave per
// row tile with its operator rows in registers; otherwise (and for the
// per-entry M2L) the streaming form with at most 8 waves in balanced passes.
template <typename R, int MODE>
void launch_trans(const TransArgs &ta, dim3 grid_items, const R *ops, const R *in, R *out,
                  int lev, hipStream_t s) {
    const int nrt = (ta.K + 15) / 16, ks = ta.KK / 4;
    // (the per-entry M2L streams its operators: measured faster there)
    if (MODE != 0 && nrt <= 8 && ks <= 32) {
        const unsigned nthr = 64u * (unsigned)nrt;
        if (ks <= 16) launch_trans_k<R, MODE, 16>(ta, grid_items, nthr, ops, in, out, lev, s);
        else if (ks <= 24) launch_trans_k<R, MODE, 24>(ta, grid_items, nthr, ops, in, out, lev, s);
        else launch_trans_k<R, MODE, 32>(ta, grid_items, nthr, ops, in, out, lev, s);
    } else {
        const int passes = (nrt + 7) / 8;
        const unsigned nthr = 64u * (unsigned)((nrt + passes - 1) / passes);
        launch_trans_k<R, MODE, 0>(ta, grid_items, nthr, ops, in, out, lev, s);
    }
}

// L[B] = sum of the M2L results of the groups of V(B), stored target-major
// as slots [ns vg_ptr[B], ns vg_ptr[B+1]) of Z (ns per group, 2 KZ values
// each: kernel 0, then kernel 1, each K values and a zero pad).  Four waves
// take every fourth slot, reading 16 bytes per lane and four slots per step;
// their partial sums are added in wave order.
template <typename R>
__global__ void __launch_bounds__(256) k_m2l_reduce(int K, int KZ, int ns, long long nbox,
                                                    const int *vptr,
                                                    const R *__restrict__ Z, R *__restrict__ L) {
    constexpr int VB = 16 / (int)sizeof(R);            // elements per 16-byte vector
    typedef R V __attribute__((ext_vector_type(VB)));
    constexpr int KZMAX = ((MAXP + 1) * (MAXP + 1) + 15) / 16 * 16;
    constexpr int NT = (2 * KZMAX / VB + 63) / 64;     // vectors per lane, at most
    __shared__ R red[4][2 * KZMAX];
    const long long box = blockIdx.x;
    if (box >= nbox) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int W = 2 * KZ, NV = W / VB;                 // KZ is a multiple of 16
    const long long q0 = (long long)ns * vptr[box], q1 = (long long)ns * vptr[box + 1];
    V acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = V{};
    long long q = q0 + wave;
    for (; q + 12 < q1; q += 16) {
        const V *z0 = reinterpret_cast<const V *>(Z + q * W);
        const V *z1 = z0 + 4 * (long long)NV, *z2 = z0 + 8 * (long long)NV;
        const V *z3 = z0 + 12 * (long long)NV;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int v = lane + 64 * t;
            if (v < NV) acc[t] += (z0[v] + z1[v]) + (z2[v] + z3[v]);
        }
    }
    for (; q < q1; q += 4) {
        const V *z0 = reinterpret_cast<const V *>(Z + q * W);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int v = lane + 64 * t;
            if (v < NV) acc[t] += z0[v];
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int v = lane + 64 * t;
        if (v < NV) *reinterpret_cast<V *>(&red[wave][v * VB]) = acc[t];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < W; i += 256) {
        const int kern = i >= KZ, k = i - kern * KZ;
        if (k < K)
            L[box * 2 * K + kern * K + k] = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
    }
}

// L2P: one block per item, wave w evaluates the local expansion of kernel w
// (potential and normal derivative) at one target point per lane, with the
// coefficients of that point's leaf.
template <typename R, int PC>
__global__ void __launch_bounds__(128) k_l2p(BasisDev B, TreeDev T, const int *pm_leaf,
                                             const int *pm_first, const int *pm_count,
                                             const R *px, const R *py, const R *pz,
                                             const R *pnx, const R *pny, const R *pnz,
                                             const R *L, long long n, R *phi, int nlev) {
    extern __shared__ __align__(16) unsigned char tab_raw[];
    const PmItem it(pm_leaf, pm_first, pm_count, T, blockIdx.x);
    const int K = B.K;
    // the item's local expansions (<= 4 leaves, both kernels) after the tables
    R *Ls = reinterpret_cast<R *>(tab_raw + basis_tab_bytes(B.P, nlev, sizeof(R)));
    for (int idx = threadIdx.x; idx < it.cnt * 2 * K; idx += blockDim.x)
        Ls[idx] = L[(long long)pm_leaf[it.first + idx / (2 * K)] * 2 * K + idx % (2 * K)];
    const BasisTab<R> tab = stage_basis<R>(B, nlev, tab_raw);   // (ends with a barrier)
    const int lane = threadIdx.x & 63;
    const int kern = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int c0 = 0; c0 < it.tot; c0 += 64) {
        const int q = c0 + lane;
        const bool ok = q < it.tot;
        const int g = it.leaf_of(ok ? q : 0);
        const int leaf = pm_leaf[it.first + g];
        const int lev = T.level[leaf];
        const int i = T.ptb[leaf] + (ok ? q - it.offs[g] : 0);
        const R cx = R(T.center[3 * leaf]), cy = R(T.center[3 * leaf + 1]);
        const R cz = R(T.center[3 * leaf + 2]);
        const R *Lb = Ls + (g * 2 + kern) * K;
        R p = R(0), dp = R(0);
        const R vx = px[i] - cx, vy = py[i] - cy, vz = pz[i] - cz;
        regular_basis_o<PC, R, Dual<R>>(B, tab, kern, lev, Dual<R>(vx, pnx[i]),
                                        Dual<R>(vy, pny[i]), Dual<R>(vz, pnz[i]),
                                        [&](int k, Dual<R> r) {
                                      const R l = Lb[k];
                                      p += l * r.v;
                                      dp += l * r.d;
                                  });
        if (ok) {
            phi[(2 * kern) * n + i] = lev >= 2 ? p : R(0);
            phi[(2 * kern + 1) * n + i] = lev >= 2 ? dp : R(0);
        }
    }
}

// ---------------------------------------------------------------------------
// W and X lists by expansions (Section 3.2: list 4 by a source-to-local
// translation, list 3 by a multipole-to-target one).  A W-list box C of leaf
// B is well separated from B at C's scale, so C's multipole converges at B's
// points (M2P), and B's points converge in C's local expansion (P2L, the X
// side).  The weighted singular basis of kernel `kern` at v from the centre
// of a box of level lev (side s, u = v / s):
//   Laplace   S_k(v) = R_k(u) |u|^-(2n+1) W_n
//   screened  S_k(v) = R_k(u) [k_n(kappa s |u|) / k_n(kappa s)] |u|^-n W_n
// with W_n the expansion weights (the translation operators sample the same
// functions): the far field of a multipole M is sum_k M_k S_k(x - c), and a
// source q at y adds q S_k(y - c) to the local expansion about c.
// ---------------------------------------------------------------------------
template <typename R> __device__ inline Dual<R> dsqrt(Dual<R> a) {
    const R r = sqrt(a.v);
    return {r, a.d / (R(2) * r)};
}
template <typename R> __device__ inline Dual<R> drcp(Dual<R> a) {
    const R r = R(1) / a.v;
    return {r, -a.d * r * r};
}
template <typename R> __device__ inline Dual<R> dexpn(Dual<R> a) {  // exp(-a)
    const R e = exp(-a.v);
    return {e, -a.d * e};
}

// The radial factors rad[n] of S_k (everything but the raw solid harmonic of
// u and its orthonormalisation factor), for compile-time order PC.  Wl[n],
// kil[n]: W_n and 1 / k_n(kappa s) of this kernel and level.
template <int PC, typename R>
__device__ inline void singular_radial(R kappa_s, const R *Wl, const R *kil, bool scr,
                                       Dual<R> ux, Dual<R> uy, Dual<R> uz, Dual<R> *rad) {
    typedef Dual<R> S;
    const S ru = dsqrt((ux * ux + uy * uy) + uz * uz);
    const S ir = drcp(ru);
    if (!scr) {
        S f = ir;
        const S ir2 = ir * ir;
#pragma unroll
        for (int n = 0; n <= PC; ++n) {
            rad[n] = f * Wl[n];
            f = f * ir2;
        }
        return;
    }
    // k_0 = e^-x / x, k_1 = e^-x (1 + x) / x^2, k_n = k_{n-2} + (2n-1)/x k_{n-1}
    const S x = ru * kappa_s;
    const S ix = drcp(x), e = dexpn(x);
    S km = e * ix, kc = (e * (x + S(R(1)))) * (ix * ix), f(R(1));
#pragma unroll
    for (int n = 0; n <= PC; ++n) {
        S kn;
        if (n == 0) {
            kn = km;
        } else if (n == 1) {
            kn = kc;
        } else {
            const S nx = km + (ix * kc) * R(2 * n - 1);
            km = kc;
            kc = nx;
            kn = kc;
        }
        rad[n] = (kn * (kil[n] * Wl[n])) * f;
        f = f * ir;
    }
}

// First order m of part i when the orders 0..P are cut into `parts` runs of
// about equal harmonic counts (part i: m in [lo(i), lo(i+1))).
constexpr int solid_part_lo(int P, int parts, int i) {
    if (i <= 0) return 0;
    if (i >= parts) return P + 1;
    const int total = (P + 1) * (P + 1);
    int acc = 0;
    for (int m = 0; m <= P; ++m) {
        if (acc * parts >= i * total) return m;
        acc += m == 0 ? P + 1 : 2 * (P - m + 1);
    }
    return P + 1;
}

// Per-level tables of one kernel in LDS: W_n and 1 / k_n(kappa s) per level,
// and the orthonormalisation factors.
template <typename R>
__device__ inline void stage_wk(const BasisDev &B, const double *weight, const double *kinv,
                                int kern, int nlev, int P, R *Wt, R *Kt, R *norm) {
    for (int i = threadIdx.x; i < nlev * (P + 1); i += blockDim.x) {
        const int lev = i / (P + 1), nn = i - lev * (P + 1);
        Wt[i] = R(weight[((long long)kern * 64 + lev) * (P + 1) + nn]);
        Kt[i] = R(kinv[i]);
    }
    for (int k = threadIdx.x; k < (P + 1) * (P + 1); k += blockDim.x) norm[k] = R(B.norm[k]);
}

// M2P: one 64-point chunk of a target leaf per block, one point per lane;
// blockIdx.y is the kernel.  For each far W box C of the leaf, C's multipole
// (times the orthonormalisation factors) is staged in LDS and evaluated at
// the lane's point, value and derivative along the point's normal; the sums
// are added to the far-field values L2P wrote.
template <typename R, int PC>
__global__ void __launch_bounds__(64) k_m2p(BasisDev B, TreeDev T, const int *__restrict__ item_leaf,
                                            const int *__restrict__ item_tb,
                                            const int *__restrict__ fw_ptr,
                                            const int *__restrict__ fw_idx, const R *px,
                                            const R *py, const R *pz, const R *pnx, const R *pny,
                                            const R *pnz, const R *__restrict__ M,
                                            const double *weight, const double *kinv, long long n,
                                            R *phi, int nlev) {
    constexpr int K = (PC + 1) * (PC + 1);
    __shared__ R Ms[K], norm[K], Wt[64 * (PC + 1)], Kt[64 * (PC + 1)];
    const int kern = blockIdx.y;
    const int leaf = item_leaf[blockIdx.x];
    const int i = item_tb[blockIdx.x] + (int)threadIdx.x;
    const bool ok = i < T.pte[leaf];
    stage_wk<R>(B, weight, kinv, kern, nlev, PC, Wt, Kt, norm);
    const bool scr = kern == 1 && B.screened;
    const int ii = ok ? i : T.ptb[leaf];
    const R x = px[ii], y = py[ii], z = pz[ii];
    const R nx = pnx[ii], ny = pny[ii], nz = pnz[ii];
    R p = R(0), dp = R(0);
    for (int q = fw_ptr[leaf]; q < fw_ptr[leaf + 1]; ++q) {
        const int C = fw_idx[q];
        __syncthreads();                               // tables staged / last box read
        for (int k = threadIdx.x; k < K; k += 64)
            Ms[k] = M[((long long)C * 2 + kern) * K + k] * norm[k];
        __syncthreads();
        const int lev = T.level[C];
        const R is = R(1.0 / B.side[lev]);
        const Dual<R> ux((x - R(T.center[3 * C])) * is, nx * is);
        const Dual<R> uy((y - R(T.center[3 * C + 1])) * is, ny * is);
        const Dual<R> uz((z - R(T.center[3 * C + 2])) * is, nz * is);
        Dual<R> rad[PC + 1];
        singular_radial<PC, R>(R(B.kappa * B.side[lev]), Wt + lev * (PC + 1),
                               Kt + lev * (PC + 1), scr, ux, uy, uz, rad);
        for_each_solid_p<PC, 0, PC, R>(ux, uy, uz, [&](int k, int nn, Dual<R> r) {
            const Dual<R> w = r * rad[nn];
            p += Ms[k] * w.v;
            dp += Ms[k] * w.d;
        });
    }
    if (ok) {
        phi[(2 * kern) * n + i] += p;
        phi[(2 * kern + 1) * n + i] += dp;
    }
}

// P2L of the orders m = M0..M1: the block's 64 lanes take the points of the
// box's far X leaves in turn, each summing q S_k + (dipole) dS_k/dn of its
// points in registers; a butterfly over the wave adds the lanes, and lane 0
// adds the sums (times the orthonormalisation factors) to the box's local
// expansion.
template <typename R, int PC, int M0, int M1>
__device__ inline void p2l_range(const BasisDev &B, const TreeDev &T, const R *norm,
                                 const R *Wl, const R *kil, bool scr, int lev, int C, int kern,
                                 const int *fx_ptr, const int *fx_idx, const R *px, const R *py,
                                 const R *pz, const R *pnx, const R *pny, const R *pnz,
                                 const R *sf, const R *sh, R inv_ebar, R *Lc) {
    constexpr int K = (PC + 1) * (PC + 1);
    constexpr int KS = solid_count(PC, M0, M1);
    const R cx = R(T.center[3 * C]), cy = R(T.center[3 * C + 1]), cz = R(T.center[3 * C + 2]);
    const R is = R(1.0 / B.side[lev]), kappa_s = R(B.kappa * B.side[lev]);
    R acc[KS];
#pragma unroll
    for (int j = 0; j < KS; ++j) acc[j] = R(0);
    for (int q = fx_ptr[C]; q < fx_ptr[C + 1]; ++q) {
        const int Bl = fx_idx[q];
        for (int i = T.ptb[Bl] + (int)threadIdx.x; i < T.pte[Bl]; i += 64) {
            const R qv = sh[i], dmag = -sf[i];
            const R dip = kern == 0 ? dmag * inv_ebar : dmag;
            const Dual<R> ux((px[i] - cx) * is, pnx[i] * is), uy((py[i] - cy) * is, pny[i] * is);
            const Dual<R> uz((pz[i] - cz) * is, pnz[i] * is);
            Dual<R> rad[PC + 1];
            singular_radial<PC, R>(kappa_s, Wl, kil, scr, ux, uy, uz, rad);
            int j = 0;                                // static after unrolling
            for_each_solid_p<PC, M0, M1, R>(ux, uy, uz, [&](int, int nn, Dual<R> r) {
                const Dual<R> w = r * rad[nn];
                acc[j] += qv * w.v + dip * w.d;
                ++j;
            });
        }
    }
#pragma unroll
    for (int j = 0; j < KS; ++j) {
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) acc[j] += __shfl_xor(acc[j], o, 64);
    }
    if (threadIdx.x != 0) return;
    R *out = Lc + ((long long)C * 2 + kern) * K;
    int j = 0;
    // the same (k, n) sequence; the harmonics themselves are dead code here
    for_each_solid_p<PC, M0, M1, R>(R(0), R(0), R(0), [&](int k, int, R) {
        out[k] += acc[j] * norm[k];
        ++j;
    });
}

template <typename R, int PC, int NPART, int I>
__device__ inline void p2l_part(int part, const BasisDev &B, const TreeDev &T, const R *norm,
                                const R *Wl, const R *kil, bool scr, int lev, int C, int kern,
                                const int *fx_ptr, const int *fx_idx, const R *px, const R *py,
                                const R *pz, const R *pnx, const R *pny, const R *pnz,
                                const R *sf, const R *sh, R inv_ebar, R *Lc) {
    if constexpr (I < NPART) {
        constexpr int M0 = solid_part_lo(PC, NPART, I), M1 = solid_part_lo(PC, NPART, I + 1) - 1;
        static_assert(M0 <= M1, "empty order range");
        if (part == I)
            p2l_range<R, PC, M0, M1>(B, T, norm, Wl, kil, scr, lev, C, kern, fx_ptr, fx_idx, px,
                                     py, pz, pnx, pny, pnz, sf, sh, inv_ebar, Lc);
        else
            p2l_part<R, PC, NPART, I + 1>(part, B, T, norm, Wl, kil, scr, lev, C, kern, fx_ptr,
                                          fx_idx, px, py, pz, pnx, pny, pnz, sf, sh, inv_ebar,
                                          Lc);
    }
}

// P2L: one box with far X leaves per block, blockIdx.y the kernel, blockIdx.z
// one of NPART ranges of orders m (fewer accumulators per lane).  Runs after
// the M2L sums are in the local expansions and before L2L.
template <typename R, int PC, int NPART>
__global__ void __launch_bounds__(64) k_p2l(BasisDev B, TreeDev T, const int *__restrict__ boxes,
                                            const int *__restrict__ fx_ptr,
                                            const int *__restrict__ fx_idx, const R *px,
                                            const R *py, const R *pz, const R *pnx, const R *pny,
                                            const R *pnz, const R *sf, const R *sh, R inv_ebar,
                                            const double *weight, const double *kinv, R *Lc,
                                            int nlev) {
    constexpr int K = (PC + 1) * (PC + 1);
    __shared__ R norm[K], Wt[64 * (PC + 1)], Kt[64 * (PC + 1)];
    const int kern = blockIdx.y;
    const int C = boxes[blockIdx.x];
    stage_wk<R>(B, weight, kinv, kern, nlev, PC, Wt, Kt, norm);
    __syncthreads();
    const int lev = T.level[C];
    const bool scr = kern == 1 && B.screened;
    p2l_part<R, PC, NPART, 0>((int)blockIdx.z, B, T, norm, Wt + lev * (PC + 1),
                              Kt + lev * (PC + 1), scr, lev, C, kern, fx_ptr, fx_idx, px, py, pz,
                              pnx, pny, pnz, sf, sh, inv_ebar, Lc);
}

template <typename R>
__global__ void k_fill_zero(R *a, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = R(0);
}

}  // namespace

void build_fmm_operators(const Tree &t, const Lists &Ls, int P, double kappa, bool bf16_m2l,
                         Fmm &F, hipStream_t s) {
    require(P >= 2 && P <= MAXP, ST_INVALID, "expansion order must be in [2, 20]");
    require(t.nlev <= 64, ST_INVALID, "too many tree levels");
    F.P = P;
    F.K = (P + 1) * (P + 1);
    F.nlev = t.nlev;
    F.kappa = kappa;
    F.screened = kappa > 0.0;
    const int K = F.K, nlev = t.nlev;
    // orthonormalisation factors and 1/(2n+1)!!
    std::vector<double> norm(K), idf(P + 2);
    for (int n = 0; n <= P; ++n)
        for (int m = -n; m <= n; ++m) {
            int am = std::abs(m);
            double r = 1.0;  // (n-|m|)!/(n+|m|)!
            for (int j = n - am + 1; j <= n + am; ++j) r /= j;
            double v = (2.0 * n + 1.0) / (4.0 * M_PI) * r;
            norm[n * n + n + m] = std::sqrt(am == 0 ? v : 2.0 * v);
        }
    double df = 1.0;
    for (int n = 0; n <= P + 1; ++n) { df *= (2.0 * n + 1.0); idf[n] = 1.0 / df; }
    // recurrence coefficients of the solid harmonics and g_n series ratios
    std::vector<double> rec((size_t)2 * (P + 1) * (P + 1), 0.0), gser(2 * GSER, 0.0);
    for (int n = 0; n <= P; ++n)
        for (int m = 0; m < n; ++m) {
            rec[2 * (n * (P + 1) + m)] = (2.0 * n - 1.0) / (n - m);
            rec[2 * (n * (P + 1) + m) + 1] = (n + m - 1.0) / (n - m);
        }
    for (int row = 0; row < 2; ++row) {
        const int n = P - row;
        for (int k = 1; k < GSER; ++k) gser[row * GSER + k] = 0.5 / ((double)k * (2.0 * n + 2.0 * k + 1.0));
    }
    F.rec.alloc(rec.size()); F.rec.upload(rec.data(), rec.size(), s);
    F.gser.alloc(gser.size()); F.gser.upload(gser.data(), gser.size(), s);
    F.norm.alloc(K); F.norm.upload(norm.data(), K, s);
    F.inv_dfact.alloc(P + 2); F.inv_dfact.upload(idf.data(), P + 2, s);
    F.side.alloc(nlev); F.side.upload(t.side.data(), nlev, s);
    F.ginv.alloc((size_t)nlev * (P + 1));
    F.kinv.alloc((size_t)nlev * (P + 1));
    F.weight.alloc((size_t)2 * 64 * (P + 1));
    BasisDev B = F.dev();
    k_level_consts<<<nlev, 1, 0, s>>>(B, nlev, F.ginv.p, F.kinv.p, F.weight.p);
    KCHK();
    // quadrature on the unit sphere: Gauss-Legendre in cos(theta) x trapezoid in phi
    const int nth = (P + 57) / 2, nph = 2 * nth, Q = nth * nph;
    std::vector<double> gx(nth), gw(nth), dir(3 * Q), wq(Q);
    gauss_legendre01(nth, gx.data(), gw.data());
    for (int i = 0; i < nth; ++i) {
        double ct = 2.0 * gx[i] - 1.0, st = std::sqrt(std::fmax(0.0, 1.0 - ct * ct));
        for (int j = 0; j < nph; ++j) {
            double ph = 2.0 * M_PI * j / nph;
            int q = i * nph + j;
            dir[3 * q] = st * std::cos(ph);
            dir[3 * q + 1] = st * std::sin(ph);
            dir[3 * q + 2] = ct;
            wq[q] = 2.0 * gw[i] * (2.0 * M_PI / nph);
        }
    }
    DBuf<double> ddir(3 * Q), dwq(Q), Yw((size_t)Q * K);
    ddir.upload(dir.data(), 3 * Q, s);
    dwq.upload(wq.data(), Q, s);
    k_sphere_table<<<grid_for(Q, 128), 128, 0, s>>>(B, Q, ddir.p, dwq.p, Yw.p);
    KCHK();
    // descriptors
    std::vector<MatDesc> desc;
    F.nkey = nlev > 2 ? (long long)(nlev - 2) * 316 : 0;
    F.T.alloc((size_t)2 * std::max(F.nkey, 1ll) * K * K);
    F.Ut.alloc((size_t)2 * nlev * 8 * K * K);
    // levels without operators stay zero in the packed copies too
    F.T.zero((size_t)2 * std::max(F.nkey, 1ll) * K * K, s);
    F.Ut.zero((size_t)2 * nlev * 8 * K * K, s);
    std::vector<int> offs;  // offset class -> (dx,dy,dz)
    for (int dx = -3; dx <= 3; ++dx)
        for (int dy = -3; dy <= 3; ++dy)
            for (int dz = -3; dz <= 3; ++dz)
                if (std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz))) > 1) {
                    offs.push_back(dx); offs.push_back(dy); offs.push_back(dz);
                }
    // The Laplace operators are projected at one level only: in the level-scaled
    // bases every M2L input scales with the box side by an exact power of two
    // (offsets, sphere radius, the 1/((2n+1) s) weights), so the level-l
    // operator is the reference one times side[ref]/side[l], bit for bit; the
    // Laplace M2M / L2L operators are the same at every level.
    const int ref_lev = Ls.levels_with_v.empty() ? 2 : Ls.levels_with_v.front();
    for (int kern = 0; kern < 2; ++kern) {
        for (int lev : Ls.levels_with_v) {
            if (kern == 0 && lev != ref_lev) continue;
            double sl = t.side[lev];
            for (int c = 0; c < 316; ++c) {
                // target centre minus source centre = -offset * side
                double dx = -offs[3 * c] * sl, dy = -offs[3 * c + 1] * sl, dz = -offs[3 * c + 2] * sl;
                double rq = 0.5 * std::sqrt(dx * dx + dy * dy + dz * dz);
                long long key = (long long)(lev - 2) * 316 + c;
                desc.push_back(MatDesc{0, kern, lev, dx, dy, dz, rq,
                                       ((long long)kern * F.nkey + key) * K * K});
            }
        }
        for (int lev = 2; lev + 1 < nlev; ++lev) {
            if (kern == 0 && lev != 2) continue;
            double sc = t.side[lev + 1];
            for (int o = 0; o < 8; ++o) {
                double d[3];
                for (int a = 0; a < 3; ++a) d[a] = 0.5 * sc * (((o >> a) & 1) ? 1.0 : -1.0);
                desc.push_back(MatDesc{1, kern, lev, d[0], d[1], d[2], sc,
                                       (((long long)kern * nlev + lev) * 8 + o) * K * K});
            }
        }
    }
    const long long per = (long long)Q * K;
    const int batch = (int)std::max(1ll, std::min(256ll, (256ll << 20) / (per * 8)));
    DBuf<double> samples((size_t)batch * per), rs((size_t)batch * K);
    DBuf<MatDesc> ddesc(desc.size() + 1);
    ddesc.upload(desc.data(), desc.size(), s);
    for (size_t m0 = 0; m0 < desc.size(); m0 += batch) {
        int nb = (int)std::min<size_t>(batch, desc.size() - m0);
        k_basis_samples<<<grid_for((long long)nb * Q, 128), 128,
                          basis_tab_bytes(P, nlev, sizeof(double)), s>>>(
            B, ddesc.p + m0, nb, Q, ddir.p, F.kinv.p, F.weight.p, samples.p, rs.p, nlev);
        KCHK();
        dim3 grid((K + 63) / 64, (K + 63) / 64, nb);
        k_project_gemm<<<grid, dim3(16, 16), 0, s>>>(Yw.p, samples.p, rs.p, ddesc.p + m0, K, Q,
                                                     F.T.p, F.Ut.p);
        KCHK();
    }
    // the other levels' Laplace operators from the reference ones
    {
        const long long KK2 = (long long)K * K;
        for (int lev : Ls.levels_with_v) {
            if (lev == ref_lev) continue;
            const double f = t.side[ref_lev] / t.side[lev];   // a power of two
            k_scale_copy<<<grid_for(316 * KK2, 256), 256, 0, s>>>(
                F.T.p + (long long)(ref_lev - 2) * 316 * KK2, f, 316 * KK2,
                F.T.p + (long long)(lev - 2) * 316 * KK2);
            KCHK();
        }
        for (int lev = 3; lev + 1 < nlev; ++lev) {
            k_scale_copy<<<grid_for(8 * KK2, 256), 256, 0, s>>>(
                F.Ut.p + (long long)2 * 8 * KK2, 1.0, 8 * KK2, F.Ut.p + (long long)lev * 8 * KK2);
            KCHK();
        }
    }
    // operand-order packing (FP64 and FP32), then drop the plain copies
    F.KK = (K + 3) / 4 * 4;
    const int NRT = (K + 15) / 16;
    F.KZ = NRT * 16;
    F.PM = (long long)NRT * 16 * F.KK;
    auto pack = [&](const DBuf<double> &src, long long nmat, int transpose, DBuf<double> &d,
                    DBuf<float> &d32) {
        // tail pad: the translation kernels read up to 32 fragments of 64
        // past the start of a matrix's last row tile (values unused)
        const size_t pad = 32 * 64;
        d.alloc((size_t)nmat * F.PM + pad);
        d32.alloc((size_t)nmat * F.PM + pad);
        HIPCHK(hipMemsetAsync(d.p, 0, ((size_t)nmat * F.PM + pad) * sizeof(double), s));
        HIPCHK(hipMemsetAsync(d32.p, 0, ((size_t)nmat * F.PM + pad) * sizeof(float), s));
        k_pack<<<grid_for(nmat * F.PM, 256), 256, 0, s>>>(src.p, nmat, K, F.KK, NRT, transpose,
                                                          d.p, d32.p);
        KCHK();
    };
    pack(F.T, 2 * std::max(F.nkey, 1ll), 0, F.Tp, F.Tp32);
    pack(F.Ut, 2ll * nlev * 8, 1, F.Up, F.Up32);
    pack(F.Ut, 2ll * nlev * 8, 0, F.Lp, F.Lp32);
    if (bf16_m2l) {
        F.KC = (K + 31) / 32;
        F.PMB = (long long)NRT * F.KC * 64 * 8;
        const long long nmat = 2 * std::max(F.nkey, 1ll);
        const size_t padb = 64 * 8;   // one prefetched chunk past the last matrix
        F.Tbh.alloc((size_t)nmat * F.PMB + padb);
        F.Tbl.alloc((size_t)nmat * F.PMB + padb);
        HIPCHK(hipMemsetAsync(F.Tbh.p, 0, ((size_t)nmat * F.PMB + padb) * 2, s));
        HIPCHK(hipMemsetAsync(F.Tbl.p, 0, ((size_t)nmat * F.PMB + padb) * 2, s));
        k_pack_bf16<<<grid_for(nmat * F.PMB, 256), 256, 0, s>>>(F.T.p, nmat, K, F.KC, NRT,
                                                               F.Tbh.p, F.Tbl.p);
        KCHK();
    }
    HIPCHK(hipStreamSynchronize(s));
    F.T.release();
    F.Ut.release();
}

template <typename R> struct Ops;
template <> struct Ops<double> {
    static const double *T(const Fmm &F) { return F.Tp.p; }
    static const double *U(const Fmm &F) { return F.Up.p; }
    static const double *L(const Fmm &F) { return F.Lp.p; }
};
template <> struct Ops<float> {
    static const float *T(const Fmm &F) { return F.Tp32.p; }
    static const float *U(const Fmm &F) { return F.Up32.p; }
    static const float *L(const Fmm &F) { return F.Lp32.p; }
};

// The far-field pass shared by the matvec (one point set) and the
// right-hand side / energy (sources and targets from different sets).
template <typename R>
void far_field_pass(const Fmm &F, const Tree &t, const Lists &L, const FarSide<R> &src,
                    const R *sf, const R *sh, const FarSide<R> &dst, double inv_ebar,
                    bool clear_m, const FarWork<R> &w, Prof *prof, hipStream_t s) {
    BasisDev B = F.dev();
    TreeDev Ts{t.level.p, t.parent.p, t.child_begin.p, t.n_child.p, src.ptb, src.pte,
               t.prefix.p, t.center.p};
    TreeDev Td{t.level.p, t.parent.p, t.child_begin.p, t.n_child.p, dst.ptb, dst.pte,
               t.prefix.p, t.center.p};
    const int K = F.K;
    const long long n = dst.n;
    if (L.n_v == 0) {
        // no box has a far field: every pair is in a U/W/X list (a fill
        // kernel, not a memset, so that the matvec can be graph-captured)
        k_fill_zero<R><<<grid_for(4 * n, 256), 256, 0, s>>>(w.phi, 4 * n);
        KCHK();
        return;
    }
    if (clear_m) {
        // leaves without source points get no P2M item: zero multipoles
        k_fill_zero<R><<<grid_for(t.nbox * 2 * K, 256), 256, 0, s>>>(w.M, t.nbox * 2 * K);
        KCHK();
    }
    bool p2m_done = false;
    if (sizeof(R) == sizeof(float) && src.n_pm > 0 && src.pm_bysize) {
        // FP32, common orders: the accumulating kernel, four lanes per leaf
        // (FP64 accumulators would leave one wave per SIMD)
        constexpr int S = 4;
        auto go = [&](auto kfn, int ms) {
            ProfScope ps(prof, "p2m", s);
            const long long lanes = src.n_pm_leaves * S;
            kfn<<<dim3(blocks_ok((lanes + 255) / 256, 256), 2, ms), 256,
                  basis_tab_bytes(F.P, F.nlev, sizeof(R)), s>>>(
                B, Ts, src.pm_bysize, src.n_pm_leaves, src.ptb, src.pte, src.x, src.y, src.z,
                src.nx, src.ny, src.nz, sf, sh, R(inv_ebar), w.M, F.nlev);
            KCHK();
            p2m_done = true;
        };
        if constexpr (sizeof(R) == sizeof(float)) {
            switch (F.P) {
                case 6: go(k_p2m_acc<R, 6, S, 2>, 2); break;
                case 8: go(k_p2m_acc<R, 8, S, 2>, 2); break;
                case 10: go(k_p2m_acc<R, 10, S, 2>, 2); break;
                default: break;
            }
        }
    }
    if (src.n_pm > 0 && !p2m_done) {
        ProfScope ps(prof, "p2m", s);
        // one wave per kernel and 64-point chunk of the largest item: up to
        // four chunks at once for FP32, two for FP64, within 60 KB of LDS
        const size_t lds = basis_tab_bytes(F.P, F.nlev, sizeof(R));
        auto lds_total = [&](int nc) {
            return (size_t)nc * 2 * 16 * (65 * sizeof(R) + sizeof(int)) + lds +
                   (size_t)nc * 2 * K * sizeof(R);
        };
        int nc = (int)std::min<long long>((src.pm_max_points + 63) / 64, sizeof(R) == 4 ? 4 : 2);
        if (nc == 3) nc = 4;
        while (nc > 1 && lds_total(nc) > 60 * 1024) nc /= 2;
        auto go = [&](auto kfn, int ncb) {
            kfn<<<blocks_ok(src.n_pm, 128 * ncb), 128 * ncb, lds + (size_t)ncb * 2 * K * sizeof(R), s>>>(
                B, Ts, src.pm_leaf, src.pm_first, src.pm_count, src.x, src.y, src.z, src.nx,
                src.ny, src.nz, sf, sh, R(inv_ebar), w.M, F.nlev);
        };
        if (nc <= 1) {
            go(k_p2m<R, 1>, 1);
        } else if (nc == 2) {
            go(k_p2m<R, 2>, 2);
        } else {
            if constexpr (sizeof(R) == sizeof(float)) go(k_p2m<R, 4>, 4);
        }
        KCHK();
    }
    if (w.p2m_done) HIPCHK(hipEventRecord(w.p2m_done, s));
    TransArgs ta{};
    ta.K = K;
    ta.KK = F.KK;
    ta.KZ = F.KZ;
    ta.PM = F.PM;
    ta.nlev = F.nlev;
    ta.nkey = F.nkey;
    ta.item_ops = L.m2l_item_ops.p;
    ta.item_begin = L.m2l_item_begin.p;
    ta.item_count = L.m2l_item_count.p;
    ta.cols = L.m2l_cols.p;
    ta.vgsrc = L.m2l_grouped ? L.vg_src.p : L.v_idx.p;
    ta.vstride = L.m2l_grouped ? 8 : 1;
    ta.nsplit = L.m2l_split;
    ta.cb = t.child_begin.p;
    ta.nc = t.n_child.p;
    ta.prefix = t.prefix.p;
    {
        ProfScope ps(prof, "m2m", s);
        for (int lev = t.nlev - 2; lev >= 2; --lev) {
            ta.lb = t.level_start[lev];
            ta.le = t.level_start[lev + 1];
            ta.ncap = ta.le - ta.lb;
            launch_trans<R, 1>(ta, dim3(1, 2), Ops<R>::U(F), w.M, w.Mt, lev, s);
            k_m2m_sum<R><<<(unsigned)(ta.le - ta.lb), 64, 0, s>>>(K, ta.lb, ta.le, ta.ncap,
                                                                  t.n_child.p, w.Mt, w.M);
            KCHK();
        }
    }
    if (L.n_m2l_items > 0) {
        ProfScope ps(prof, "m2l", s);
        ta.n_items = (int)L.n_m2l_items;
        // grid padded to a multiple of 8 for the XCD-contiguous item mapping
        const unsigned gx = (unsigned)((L.n_m2l_items + 7) / 8 * 8);
        bool done = false;
        if (L.m2l_pairs && !w.bf16_m2l) {
            TransArgs tp = ta;
            tp.n_items = (int)L.n_pr_items;
            tp.item_ops = L.pr_item_ops.p;
            tp.item_begin = L.pr_item_begin.p;
            tp.item_count = L.pr_item_count.p;
            tp.pr_src = L.pr_src.p;
            tp.pr_slot = L.pr_slot.p;
            const unsigned gp = (unsigned)((L.n_pr_items + 7) / 8 * 8);
            done = gp > 0 && launch_m2l_pairs<R>(tp, gp, Ops<R>::T(F), w.M, w.Z, s);
        }
        if (done) {
        } else if constexpr (sizeof(R) == sizeof(float)) {
            if (w.bf16_m2l) {
                ta.KC = F.KC;
                ta.PMB = F.PMB;
                launch_m2l_bf16(ta, gx, L.m2l_grouped, reinterpret_cast<const u16x8_t *>(F.Tbh.p),
                                reinterpret_cast<const u16x8_t *>(F.Tbl.p), w.M, w.Z, s);
            } else if (L.m2l_grouped) {
                launch_m2l<R>(ta, gx, Ops<R>::T(F), w.M, w.Z, s);
            } else {
                launch_trans<R, 0>(ta, dim3(gx, 2), Ops<R>::T(F), w.M, w.Z, 0, s);
            }
        } else if (L.m2l_grouped) {
            launch_m2l<R>(ta, gx, Ops<R>::T(F), w.M, w.Z, s);
        } else {
            launch_trans<R, 0>(ta, dim3(gx, 2), Ops<R>::T(F), w.M, w.Z, 0, s);
        }
    }
    {
        ProfScope ps(prof, "m2l_reduce", s);
        k_m2l_reduce<R><<<blocks_ok(t.nbox, 256), 256, 0, s>>>(
            K, F.KZ, L.m2l_split, t.nbox, L.m2l_grouped ? L.vg_ptr.p : L.v_ptr.p, w.Z, w.Lc);
        KCHK();
    }
    if (L.n_p2l_boxes > 0) {
        // far X leaves into the local expansions (single-tree lists only:
        // source and target sides are the same points)
        ProfScope ps(prof, "p2l", s);
        auto go = [&](auto kfn, int np) {
            kfn<<<dim3((unsigned)L.n_p2l_boxes, 2, np), 64, 0, s>>>(
                B, Td, L.p2l_box.p, L.fx_ptr.p, L.fx_idx.p, src.x, src.y, src.z, src.nx, src.ny,
                src.nz, sf, sh, R(inv_ebar), F.weight.p, F.kinv.p, w.Lc, F.nlev);
            KCHK();
        };
        constexpr bool f32 = sizeof(R) == sizeof(float);
        switch (F.P) {
            case 6: go(k_p2l<R, 6, 2>, 2); break;
            case 8: go(k_p2l<R, 8, f32 ? 2 : 4>, f32 ? 2 : 4); break;
            case 10: go(k_p2l<R, 10, f32 ? 2 : 4>, f32 ? 2 : 4); break;
            case 14: go(k_p2l<R, 14, f32 ? 4 : 6>, f32 ? 4 : 6); break;
            default: throw Error(ST_INVALID, "W/X expansions need order 6, 8, 10 or 14");
        }
    }
    {
        ProfScope ps(prof, "l2l", s);
        for (int lev = 2; lev + 1 < t.nlev; ++lev) {
            ta.lb = t.level_start[lev];
            ta.le = t.level_start[lev + 1];
            launch_trans<R, 2>(ta, dim3(1, 2), Ops<R>::L(F), w.Lc, w.Lc, lev, s);
        }
    }
    if (dst.n_pm > 0) {
        ProfScope ps(prof, "l2p", s);
        const size_t l2p_lds = basis_tab_bytes(F.P, F.nlev, sizeof(R)) + 4 * 2 * K * sizeof(R);
        // common orders run with a compile-time recurrence (static indices,
        // constant coefficients), others with the generic table recurrence
        auto go = [&](auto kfn) {
            kfn<<<blocks_ok(dst.n_pm, 128), 128, l2p_lds, s>>>(
                B, Td, dst.pm_leaf, dst.pm_first, dst.pm_count, dst.x, dst.y, dst.z, dst.nx,
                dst.ny, dst.nz, w.Lc, n, w.phi, F.nlev);
        };
        switch (F.P) {
            case 6: go(k_l2p<R, 6>); break;
            case 8: go(k_l2p<R, 8>); break;
            case 10: go(k_l2p<R, 10>); break;
            case 14: go(k_l2p<R, 14>); break;
            default: go(k_l2p<R, 0>); break;
        }
        KCHK();
    }
    if (L.n_m2p_items > 0) {
        // far W boxes at the leaves' points, added to the L2P values
        ProfScope ps(prof, "m2p", s);
        auto go = [&](auto kfn) {
            kfn<<<dim3((unsigned)L.n_m2p_items, 2), 64, 0, s>>>(
                B, Td, L.m2p_leaf.p, L.m2p_tb.p, L.fw_ptr.p, L.fw_idx.p, dst.x, dst.y, dst.z,
                dst.nx, dst.ny, dst.nz, w.M, F.weight.p, F.kinv.p, n, w.phi, F.nlev);
            KCHK();
        };
        switch (F.P) {
            case 6: go(k_m2p<R, 6>); break;
            case 8: go(k_m2p<R, 8>); break;
            case 10: go(k_m2p<R, 10>); break;
            case 14: go(k_m2p<R, 14>); break;
            default: throw Error(ST_INVALID, "W/X expansions need order 6, 8, 10 or 14");
        }
    }
}

template <typename R>
void far_field(const Fmm &F, const Tree &t, const Lists &L, const NodeSoA &nd, const R *px,
               const R *py, const R *pz, const R *pnx, const R *pny, const R *pnz, const R *sf,
               const R *sh, double inv_ebar, long long n, const FarWork<R> &w, Prof *prof,
               hipStream_t s) {
    (void)nd;
    FarSide<R> side;
    side.ptb = t.pt_begin.p;
    side.pte = t.pt_end.p;
    side.pm_leaf = L.pm_leaf.p;
    side.pm_first = L.pm_first.p;
    side.pm_count = L.pm_count.p;
    side.n_pm = L.n_pm;
    side.pm_max_points = L.pm_max_points;
    side.pm_bysize = L.pm_bysize.p;
    side.n_pm_leaves = L.n_pm_leaves;
    side.x = px; side.y = py; side.z = pz;
    side.nx = pnx; side.ny = pny; side.nz = pnz;
    side.n = n;
    far_field_pass(F, t, L, side, sf, sh, side, inv_ebar, false, w, prof, s);
}

template <typename R>
void far_field_sides(const Fmm &F, const Tree &t, const Lists &L, const FarSide<R> &src,
                     const R *sf, const R *sh, const FarSide<R> &dst, double inv_ebar,
                     const FarWork<R> &w, Prof *prof, hipStream_t s) {
    far_field_pass(F, t, L, src, sf, sh, dst, inv_ebar, true, w, prof, s);
}

template void far_field_sides<double>(const Fmm &, const Tree &, const Lists &,
                                      const FarSide<double> &, const double *, const double *,
                                      const FarSide<double> &, double, const FarWork<double> &,
                                      Prof *, hipStream_t);
template void far_field<double>(const Fmm &, const Tree &, const Lists &, const NodeSoA &,
                                const double *, const double *, const double *, const double *,
                                const double *, const double *, const double *, const double *,
                                double, long long, const FarWork<double> &, Prof *, hipStream_t);
template void far_field<float>(const Fmm &, const Tree &, const Lists &, const NodeSoA &,
                               const float *, const float *, const float *, const float *,
                               const float *, const float *, const float *, const float *,
                               double, long long, const FarWork<float> &, Prof *, hipStream_t);

}  // namespace afmpb

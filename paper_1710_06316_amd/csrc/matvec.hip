// Near field and assembly of the matvec y = M x of Eq. (5) (Section 2):
//   P2P  -- point-rule pairs of the U, W and X lists (t != p), all four
//           kernels of Eq. (6) in cancellation-free difference form;
//   near -- patch-minus-point corrections of the near set ("four
//           multiplications" per pair);
//   combine -- y_f = alpha f + P2P_f - Phi_L + Phi_Y + near_f,
//              y_h = alpha h + P2P_h - dPhi_L/dn + dPhi_Y/dn / ebar + near_h.
#include "kernels.h"
#include "matvec.h"
#include "prof.h"

namespace afmpb {

namespace {

// Two-sum compensated accumulator (used for single precision).
template <typename R>
struct CompSum {
    R s = R(0), c = R(0);
    __device__ void add(R v) {
        R t = s + v;
        R bp = t - s;
        c += (s - (t - bp)) + (v - bp);
        s = t;
    }
    __device__ R value() const { return s + c; }
};

template <typename R>
__global__ void __launch_bounds__(64) k_p2p(const int *__restrict__ item_leaf,
                                            const int *__restrict__ item_begin,
                                            const int *__restrict__ leaf_ids,
                                            const int *__restrict__ src_ptr,
                                            const int *__restrict__ src_box,
                                            const int *__restrict__ ptb, const int *__restrict__ pte,
                                            NodeR<R> nd, const R *__restrict__ sf,
                                            const R *__restrict__ sh, R kappa, R inv_ebar,
                                            R *__restrict__ out_f, R *__restrict__ out_h) {
    __shared__ R S[8][64];
    const int w = blockIdx.x, lane = threadIdx.x;
    const int li = item_leaf[w];
    const int box = leaf_ids[li];
    const int i = item_begin[w] + lane;
    const bool act = i < pte[box];
    const R x = act ? nd.x[i] : R(0), y = act ? nd.y[i] : R(0), z = act ? nd.z[i] : R(0);
    const R n0x = act ? nd.nx[i] : R(0), n0y = act ? nd.ny[i] : R(0), n0z = act ? nd.nz[i] : R(0);
    CompSum<R> af, ah;
    for (int q = src_ptr[li]; q < src_ptr[li + 1]; ++q) {
        const int C = src_box[q];
        const int cb = ptb[C], ce = pte[C];
        for (int s0 = cb; s0 < ce; s0 += 64) {
            const int j = s0 + lane;
            __syncthreads();
            if (j < ce) {
                S[0][lane] = nd.x[j]; S[1][lane] = nd.y[j]; S[2][lane] = nd.z[j];
                S[3][lane] = nd.nx[j]; S[4][lane] = nd.ny[j]; S[5][lane] = nd.nz[j];
                S[6][lane] = sf[j]; S[7][lane] = sh[j];
            }
            __syncthreads();
            const int cnt = min(64, ce - s0);
            if (act) {
                for (int jj = 0; jj < cnt; ++jj) {
                    if (s0 + jj == i) continue;
                    Abcd<R> k = abcd_point(x - S[0][jj], y - S[1][jj], z - S[2][jj], n0x, n0y,
                                           n0z, S[3][jj], S[4][jj], S[5][jj], kappa, inv_ebar);
                    const R f = S[6][jj], h = S[7][jj];
                    af.add(k.B * f - k.A * h);
                    ah.add(k.D * f - k.C * h);
                }
            }
        }
    }
    if (act) {
        out_f[i] = af.value();
        out_h[i] = ah.value();
    }
}

template <typename R>
__global__ void k_gather_sources(const double *__restrict__ x, const double *__restrict__ area,
                                 long long n, R *sf, R *sh) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    sf[i] = R(area[i] * x[i]);
    sh[i] = R(area[i] * x[n + i]);
}

// One group of 8 lanes per row for the near correction; the row's result is
// combined with every other part of the matvec.
template <typename R>
__global__ void k_combine(long long n, const double *__restrict__ x, const R *__restrict__ pf,
                          const R *__restrict__ ph, const R *__restrict__ phi,
                          const long long *__restrict__ nptr, const int *__restrict__ ncol,
                          const double *__restrict__ nd, double alpha, double inv_ebar,
                          double *__restrict__ y) {
    long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long p = gid >> 3;
    int sub = (int)(gid & 7);
    double cf = 0.0, ch = 0.0;
    if (p < n) {
        for (long long e = nptr[p] + sub; e < nptr[p + 1]; e += 8) {
            int t = ncol[e];
            double f = x[t], h = x[n + t];
            const double *d = nd + 4 * e;
            cf += d[1] * f - d[0] * h;
            ch += d[3] * f - d[2] * h;
        }
    }
#pragma unroll
    for (int o = 4; o > 0; o >>= 1) {
        cf += __shfl_xor(cf, o, 8);
        ch += __shfl_xor(ch, o, 8);
    }
    if (p < n && sub == 0) {
        double far_f = -(double)phi[p] + (double)phi[2 * n + p];
        double far_h = -(double)phi[n + p] + inv_ebar * (double)phi[3 * n + p];
        y[p] = alpha * x[p] + (double)pf[p] + far_f + cf;
        y[n + p] = alpha * x[n + p] + (double)ph[p] + far_h + ch;
    }
}

__global__ void k_to_morton(const double *__restrict__ in, const int *__restrict__ perm,
                            long long n, double *__restrict__ out) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    long long o = perm[i];
    out[i] = in[o];
    out[n + i] = in[n + o];
}

__global__ void k_from_morton(const double *__restrict__ in, const int *__restrict__ perm,
                              long long n, double *__restrict__ out) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    long long o = perm[i];
    out[o] = in[i];
    out[n + o] = in[n + i];
}

}  // namespace

void to_morton(const double *in, const int *perm, long long n, double *out, hipStream_t s) {
    k_to_morton<<<grid_for(n, 256), 256, 0, s>>>(in, perm, n, out);
    KCHK();
}
void from_morton(const double *in, const int *perm, long long n, double *out, hipStream_t s) {
    k_from_morton<<<grid_for(n, 256), 256, 0, s>>>(in, perm, n, out);
    KCHK();
}

template <typename R>
void apply_operator(const MatvecPlan<R> &mp, const double *x, double *y, Prof *prof,
                    hipStream_t s) {
    const long long n = mp.n;
    {
        ProfScope ps(prof, "gather", s);
        k_gather_sources<R><<<grid_for(n, 256), 256, 0, s>>>(x, mp.area, n, mp.sf, mp.sh);
        KCHK();
    }
    far_field<R>(*mp.fmm, *mp.tree, *mp.lists, mp.nd64, mp.nd.x, mp.nd.y, mp.nd.z, mp.nd.nx,
                 mp.nd.ny, mp.nd.nz, mp.sf, mp.sh, mp.inv_ebar, n, mp.far, prof, s);
    {
        ProfScope ps(prof, "p2p", s);
        const Lists &L = *mp.lists;
        k_p2p<R><<<(unsigned)L.n_items, 64, 0, s>>>(L.item_box.p, L.item_begin.p, L.leaf_ids.p,
                                                    L.p2p_ptr.p, L.p2p_src.p, mp.tree->pt_begin.p,
                                                    mp.tree->pt_end.p, mp.nd, mp.sf, mp.sh,
                                                    R(mp.kappa), R(mp.inv_ebar), mp.pf, mp.ph);
        KCHK();
    }
    {
        ProfScope ps(prof, "near_combine", s);
        k_combine<R><<<grid_for(8 * n, 256), 256, 0, s>>>(n, x, mp.pf, mp.ph, mp.far.phi,
                                                          mp.near->ptr.p, mp.near->col.p,
                                                          mp.near->delta.p, mp.alpha,
                                                          mp.inv_ebar, y);
        KCHK();
    }
}

template void apply_operator<double>(const MatvecPlan<double> &, const double *, double *,
                                     Prof *, hipStream_t);
template void apply_operator<float>(const MatvecPlan<float> &, const double *, double *,
                                    Prof *, hipStream_t);

}  // namespace afmpb

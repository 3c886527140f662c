// Near field and assembly of the matvec y = M x of Eq. (5) (Section 2):
//   P2P  -- point-rule pairs of the U, W and X lists (t != p), all four
//           kernels of Eq. (6) in cancellation-free difference form;
//   near -- patch-minus-point corrections of the near set ("four
//           multiplications" per pair);
//   combine -- y_f = alpha f + P2P_f - Phi_L + Phi_Y + near_f,
//              y_h = alpha h + P2P_h - dPhi_L/dn + dPhi_Y/dn / ebar + near_h.
#include <type_traits>

#include "kernels.h"
#include "matvec.h"
#include "prof.h"

namespace afmpb {

namespace {

// Per-pair arithmetic of the P2P kernel.  The 1/(4 pi) factor is applied to
// the final sums.  1 - e^{-s}, a(s), b(s) come from their Taylor series below
// s = 0.1, from e^{-s} above (no cancellation either way).
template <typename R> struct Fast;
template <> struct Fast<double> {
    // hardware reciprocal square root refined by two Newton steps
    static __device__ inline double rsq(double x) {
        double y = __builtin_amdgcn_rsq(x);
        y = y * (1.5 - 0.5 * x * y * y);
        return y * (1.5 - 0.5 * x * y * y);
    }
    static __device__ inline double ex(double x) { return exp(x); }
    static constexpr int NSER = 10;
};
template <> struct Fast<float> {
    static __device__ inline float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ inline float ex(float x) { return __expf(x); }
    static constexpr int NSER = 6;
};

// Taylor coefficients of om(s) = 1 - e^{-s} and a(s) (see kernels.h)
struct P2PSeries {
    double om[11], a[11];
    constexpr P2PSeries() : om(), a() {
        double fact = 1.0;
        for (int k = 1; k <= 10; ++k) {
            fact *= k;
            double sg = (k & 1) ? -1.0 : 1.0;
            om[k] = -sg / fact;
            a[k] = (k >= 2) ? sg * (k - 1) / fact : 0.0;
        }
    }
};

// One wave per work chunk: <= 64 targets of one leaf against the chunk's
// source point ranges.  A group of <= 32 (16, 8) targets runs as 2 (4, 8)
// copies of 32 (16, 8) lanes, copy r taking sources r, r+f, r+2f, ... of each
// staged tile, so that small leaves still fill the wave.  Sources are staged
// 64 at a time in LDS (coalesced loads, zero fill past the range); the copies
// are added in copy order and the chunk's partial sums go to part[chunk][2][64],
// which k_p2p_reduce adds per target in chunk order (deterministic).
// A reverse chunk (rev[c] >= 0) also evaluates every pair the other way: at
// step k lane (copy q, target ti) meets source row q + f ((ti + k) mod W), so
// the lanes of one step touch distinct rows, whose sums over the tile go to
// the reverse slots rev[c] + (stream position) of rpart[slot][2].
// FP64: at least 3 waves per SIMD (168 VGPRs; left free, the compiler takes
// 174, which leaves room for only 2).
template <typename R>
__global__ void __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 1 : 3))) k_p2p(
    const int *__restrict__ ch_lo, const int *__restrict__ ch_hi, const int *__restrict__ ch_grp,
    const int *__restrict__ grp_tbeg, const int *__restrict__ grp_tend,
    const int *__restrict__ rng_b, const int *__restrict__ rng_e, const int *__restrict__ rev,
    NodeR<R> nd, const R *__restrict__ sf, const R *__restrict__ sh, R kappa, R inv_ebar,
    double *__restrict__ part, double *__restrict__ rpart) {
    constexpr P2PSeries S;
    __shared__ R T[64][8];
    // reverse sums of the tile's sources, even and odd steps apart (the two
    // updates of one trip cannot alias, so they overlap)
    __shared__ R RV0[64][2], RV1[64][2];
    __shared__ double red[2][64];
    const int lane = threadIdx.x;
    const int c = blockIdx.x;
    const int g = ch_grp[c];
    const int tb = grp_tbeg[g], te = grp_tend[g];
    const int f = p2p_replicas(te - tb);              // uniform for the wave
    const int W = 64 / f, rep = lane / W, ti = lane % W;
    const int i = tb + ti;
    const bool act = i < te;
    const int ii = act ? i : tb;
    const R x = nd.x[ii], y = nd.y[ii], z = nd.z[ii];
    const R n0x = nd.nx[ii], n0y = nd.ny[ii], n0z = nd.nz[ii];
    // this lane's target as a source of the reverse pairs (zero when inactive)
    const R tsf = act ? sf[ii] : R(0), tsh = act ? sh[ii] : R(0);
    const int roff = rev[c];                          // uniform; -1: one-directional
    double af = 0.0, ah = 0.0;
    // one source pair (T row jj) against this lane's target, added to bf, bh
    // (and, BOTH, the pair the other way to rf, rh); MASKED: the pair may be
    // the target itself or past the tile (then it adds nothing)
    auto pair = [&](auto masked, auto both, int jj, bool ok, R &bf, R &bh, R &rf, R &rh) {
        constexpr bool MASKED = decltype(masked)::value, BOTH = decltype(both)::value;
        const R rx = x - T[jj][0], ry = y - T[jj][1], rz = z - T[jj][2];
        const R snx = T[jj][3], sny = T[jj][4], snz = T[jj][5];
        const R sfv = T[jj][6], shv = T[jj][7];
        R r2 = (rx * rx + ry * ry) + rz * rz;
        if constexpr (MASKED) r2 = ok ? r2 : R(1);
        const R ir = Fast<R>::rsq(r2);
        const R rr = r2 * ir;
        const R s = kappa * rr;
        const R e = Fast<R>::ex(-s);
        R om, fa;
        if (s < R(0.1)) {
            constexpr int N = Fast<R>::NSER;
            R po = R(S.om[N]), pa = R(S.a[N]);
#pragma unroll
            for (int k = N - 1; k >= 2; --k) {
                po = po * s + R(S.om[k]);
                pa = pa * s + R(S.a[k]);
            }
            om = (po * s + R(1)) * s;
            fa = pa * s * s;
        } else {
            om = R(1) - e;
            fa = om - s * e;
        }
        // b(s) = 3 a(s) - s^2 e outside the divergent branch: the two terms
        // cancel to about a third of 3 a(s) as s -> 0 (b ~ s^2/2, a ~ s^2/2),
        // so b keeps a relative error of a few times that of a
        const R fb = R(3) * fa - (s * s) * e;
        const R Rn = (rx * snx + ry * sny) + rz * snz;
        const R Rn0 = (rx * n0x + ry * n0y) + rz * n0z;
        const R n0n = (n0x * snx + n0y * sny) + n0z * snz;
        const R ir2 = ir * ir;
        const R ir3 = ir2 * ir;
        const R e1 = e * (R(1) + s);
        const R A = om * ir;
        // B = Rn Pb, Cc = Rn0 Pc (the factors are shared with the pair the
        // other way); Pb = ir3 (1/ebar - e1), Pc = ir3 (e1/ebar - 1), one
        // fused multiply-add each
        const R ir3e = inv_ebar * ir3;
        const R Pb = ir3e - ir3 * e1;
        const R Pc = e1 * ir3e - ir3;
        const R B = Rn * Pb;
        const R Cc = Rn0 * Pc;
        const R D = ir3e * (n0n * fa - (Rn0 * Rn) * (fb * ir2));
        // the terms are added one at a time (two fused multiply-adds each)
        if constexpr (MASKED) {
            bf = ok ? (bf + B * sfv) - A * shv : bf;
            bh = ok ? (bh + D * sfv) - Cc * shv : bh;
        } else {
            bf = (bf + B * sfv) - A * shv;
            bh = (bh + D * sfv) - Cc * shv;
        }
        if constexpr (BOTH) {
            // the pair the other way, added to rf, rh: r -> -r swaps the roles
            // of the two normals (Rn -> -Rn0, Rn0 -> -Rn); A and D are unchanged
            const R Br = -Rn0 * Pb;
            const R Cr = -Rn * Pc;
            if (!MASKED || ok) {
                rf = (rf + Br * tsf) - A * tsh;
                rh = (rh + D * tsf) - Cr * tsh;
            }
        }
    };
    // Source tiles of 64 points, walked over the chunk's ranges; the next
    // tile is loaded into registers while the current one is evaluated.
    int r = ch_lo[c];
    const int rhi = ch_hi[c];
    int cb = 0, ce = 0, s0 = 0;
    if (r < rhi) { cb = rng_b[r]; ce = rng_e[r]; s0 = cb; }
    R v[8];
    auto fetch = [&](int s0n, int cen) {
        const int j = s0n + lane;
        const bool in = j < cen;
        v[0] = in ? nd.x[j] : R(0);  v[1] = in ? nd.y[j] : R(0);
        v[2] = in ? nd.z[j] : R(0);  v[3] = in ? nd.nx[j] : R(0);
        v[4] = in ? nd.ny[j] : R(0); v[5] = in ? nd.nz[j] : R(0);
        v[6] = in ? sf[j] : R(0);    v[7] = in ? sh[j] : R(0);
    };
    if (r < rhi) fetch(s0, ce);
    int pos = 0;                                      // stream position of the tile
    R rdum0, rdum1;
    while (r < rhi) {
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < 8; ++q) T[lane][q] = v[q];
        RV0[lane][0] = R(0);
        RV0[lane][1] = R(0);
        RV1[lane][0] = R(0);
        RV1[lane][1] = R(0);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int cnt = min(64, ce - s0), s0c = s0;
        // next tile (uniform): the rest of this range, else the next range
        s0 += 64;
        if (s0 >= ce) {
            ++r;
            if (r < rhi) { cb = rng_b[r]; ce = rng_e[r]; s0 = cb; }
        }
        if (r < rhi) fetch(s0, ce);
        R bf = R(0), bh = R(0);
        // two sources per trip, added in source order; jb + rep <= 63 (jb is a
        // multiple of f below cnt <= 64 and f | 64); the second row index is
        // clamped into the tile when it is past cnt (then masked).  A full
        // tile that holds none of the group's targets needs no mask (the
        // lanes past the group's targets are discarded by the reduction).
        if (roff >= 0) {                                          // uniform
            // reverse chunk (sources never include the group's targets);
            // inactive lanes add nothing the other way (zero strengths)
            auto rot = [&](auto masked, int k, R (*RV)[2]) {
                const int jrow = rep + f * ((ti + k) & (W - 1));
                R rf = RV[jrow][0], rh = RV[jrow][1];
                pair(masked, std::true_type{}, jrow, jrow < cnt, bf, bh, rf, rh);
                RV[jrow][0] = rf;
                RV[jrow][1] = rh;
            };
            if (cnt == 64) {
                for (int k = 0; k < W; k += 2) {
                    rot(std::false_type{}, k, RV0);
                    rot(std::false_type{}, k + 1, RV1);
                }
            } else {
                for (int k = 0; k < W; k += 2) {
                    rot(std::true_type{}, k, RV0);
                    rot(std::true_type{}, k + 1, RV1);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (lane < cnt) {
                double *o = rpart + 2 * ((long long)roff + pos + lane);
                o[0] = (double)(RV0[lane][0] + RV1[lane][0]);
                o[1] = (double)(RV0[lane][1] + RV1[lane][1]);
            }
        } else if (cnt == 64 && (s0c >= te || s0c + 64 <= tb)) { // uniform
            for (int jb = 0; jb < 64; jb += 2 * f) {
                pair(std::false_type{}, std::false_type{}, jb + rep, true, bf, bh, rdum0, rdum1);
                pair(std::false_type{}, std::false_type{}, jb + f + rep, true, bf, bh, rdum0, rdum1);
            }
        } else {
            for (int jb = 0; jb < cnt; jb += 2 * f) {
                const int ja = jb + rep, jc = jb + f + rep;
                const bool oka = act && ja < cnt && s0c + ja != i;
                const bool okc = act && jc < cnt && s0c + jc != i;
                pair(std::true_type{}, std::false_type{}, ja, oka, bf, bh, rdum0, rdum1);
                pair(std::true_type{}, std::false_type{}, min(jc, 63), okc, bf, bh, rdum0, rdum1);
            }
        }
        pos += cnt;
        af += (double)bf;
        ah += (double)bh;
    }
    red[0][lane] = af;
    red[1][lane] = ah;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double tf = 0.0, th = 0.0;
    if (lane < W) {
        for (int q = 0; q < f; ++q) {
            tf += red[0][q * W + lane];
            th += red[1][q * W + lane];
        }
    }
    part[((long long)c * 2) * 64 + lane] = tf;
    part[((long long)c * 2 + 1) * 64 + lane] = th;
}

__global__ void __launch_bounds__(64) k_p2p_reduce(const int *__restrict__ grp_ptr,
                                                   const int *__restrict__ grp_tbeg,
                                                   const int *__restrict__ grp_tend,
                                                   const double *__restrict__ part,
                                                   const int *__restrict__ rev_ptr,
                                                   const int *__restrict__ rev_idx,
                                                   const double *__restrict__ rpart,
                                                   double *__restrict__ out_f,
                                                   double *__restrict__ out_h, int add) {
    const int g = blockIdx.x, lane = threadIdx.x;
    const int i = grp_tbeg[g] + lane;
    if (i >= grp_tend[g]) return;
    // loads are issued RB entries ahead of the additions, which stay in
    // chunk order (few waves per SIMD: the sum is bound by load latency)
    constexpr int RB = 8;
    double tf = 0.0, th = 0.0;
    int c = grp_ptr[g];
    const int c1 = grp_ptr[g + 1];
    for (; c + RB <= c1; c += RB) {
        double vf[RB], vh[RB];
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            vf[k] = part[((long long)(c + k) * 2) * 64 + lane];
            vh[k] = part[((long long)(c + k) * 2 + 1) * 64 + lane];
        }
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            tf += vf[k];
            th += vh[k];
        }
    }
    for (; c < c1; ++c) {
        tf += part[((long long)c * 2) * 64 + lane];
        th += part[((long long)c * 2 + 1) * 64 + lane];
    }
    // the pairs evaluated the other way, in chunk order
    int q = rev_ptr[i];
    const int q1 = rev_ptr[i + 1];
    for (; q + RB <= q1; q += RB) {
        long long sl[RB];
        double vf[RB], vh[RB];
#pragma unroll
        for (int k = 0; k < RB; ++k) sl[k] = rev_idx[q + k];
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            vf[k] = rpart[2 * sl[k]];
            vh[k] = rpart[2 * sl[k] + 1];
        }
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            tf += vf[k];
            th += vh[k];
        }
    }
    for (; q < q1; ++q) {
        const long long sl = rev_idx[q];
        tf += rpart[2 * sl];
        th += rpart[2 * sl + 1];
    }
    // add: the near-set correction is already there.  The product is rounded
    // before the addition (no fused multiply-add), so that both schedules
    // add the same two rounded terms.
    {
#pragma clang fp contract(off)
        const double vf = tf * INV_4PI, vh = th * INV_4PI;
        out_f[i] = add ? out_f[i] + vf : vf;
        out_h[i] = add ? out_h[i] + vh : vh;
    }
}

// Source strengths a f, a h of every node, and (f, h) side by side in the
// working precision for the near correction's gathers.
template <typename R>
__global__ void k_gather_sources(const double *__restrict__ x, const double *__restrict__ area,
                                 long long n, R *sf, R *sh, R *xp) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double f = x[i], h = x[n + i];
    sf[i] = R(area[i] * f);
    sh[i] = R(area[i] * h);
    xp[2 * i] = R(f);
    xp[2 * i + 1] = R(h);
}

typedef float fvec4 __attribute__((ext_vector_type(4)));
typedef double dvec2 __attribute__((ext_vector_type(2)));

template <typename R> struct Pair2;
template <> struct Pair2<float> { typedef float2 T; };
template <> struct Pair2<double> { typedef double2 T; };

// Near correction: one group of 16 lanes per row, NEAR_INFLIGHT entries in
// flight per lane.  The coefficients and column indices are read once
// (non-temporal loads, so that they do not evict the gathered (f, h) pairs
// from cache); products and sums are in FP64 (a product of two FP32 values
// is exact there).  Lane partial sums are added by a fixed butterfly; the
// row's sums are added to the P2P sums (ADD) or stored for P2P to add to.
// Two entries in flight measured faster than four or eight on the 9.7M-node
// shell (13.0 / 14.4 / 13.6 ms): the dependent (f, h) gathers, not the
// streamed coefficients, bound this kernel.
#ifndef NEAR_INFLIGHT
#define NEAR_INFLIGHT 2
#endif
template <typename R, bool ADD>
__global__ void __launch_bounds__(256) k_near_apply(
    long long n, const typename Pair2<R>::T *__restrict__ xp, const long long *__restrict__ nptr,
    const int *__restrict__ ncol, const R *__restrict__ nd, double *__restrict__ pf,
    double *__restrict__ ph) {
    typedef typename Pair2<R>::T P2;
    constexpr int IN = NEAR_INFLIGHT;
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long p = gid >> 4;
    const int sub = (int)(gid & 15);
    double cf[IN], ch[IN];
#pragma unroll
    for (int q = 0; q < IN; ++q) cf[q] = ch[q] = 0.0;
    auto term = [&](int q, long long e, int t) {
        const P2 v = xp[t];
        R d[4];
        if constexpr (sizeof(R) == sizeof(float)) {
            const fvec4 c = __builtin_nontemporal_load(reinterpret_cast<const fvec4 *>(nd + 4 * e));
            d[0] = c.x; d[1] = c.y; d[2] = c.z; d[3] = c.w;
        } else {
            const dvec2 c0 = __builtin_nontemporal_load(reinterpret_cast<const dvec2 *>(nd + 4 * e));
            const dvec2 c1 = __builtin_nontemporal_load(reinterpret_cast<const dvec2 *>(nd + 4 * e + 2));
            d[0] = c0.x; d[1] = c0.y; d[2] = c1.x; d[3] = c1.y;
        }
        const double f = (double)v.x, h = (double)v.y;
        cf[q] += (double)d[1] * f - (double)d[0] * h;
        ch[q] += (double)d[3] * f - (double)d[2] * h;
    };
    if (p < n) {
        const long long e1 = nptr[p + 1];
        long long e = nptr[p] + sub;
        for (; e + 16 * (IN - 1) < e1; e += 16 * IN) {
            int t[IN];
#pragma unroll
            for (int q = 0; q < IN; ++q) t[q] = __builtin_nontemporal_load(ncol + e + 16 * q);
#pragma unroll
            for (int q = 0; q < IN; ++q) term(q, e + 16 * q, t[q]);
        }
        // fewer than IN entries left for this lane
#pragma unroll
        for (int q = 0; q < IN - 1; ++q)
            if (e + 16 * q < e1) term(q, e + 16 * q, __builtin_nontemporal_load(ncol + e + 16 * q));
    }
    double sf = 0.0, sh = 0.0;
#pragma unroll
    for (int q = 0; q < IN; ++q) {
        sf += cf[q];
        sh += ch[q];
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
        sf += __shfl_xor(sf, o, 16);
        sh += __shfl_xor(sh, o, 16);
    }
    if (p < n && sub == 0) {
        pf[p] = ADD ? pf[p] + sf : sf;
        ph[p] = ADD ? ph[p] + sh : sh;
    }
}

// y = alpha x + (P2P + near) - far field of Eq. (5).
template <typename R>
__global__ void k_combine(long long n, const double *__restrict__ x, const double *__restrict__ pf,
                          const double *__restrict__ ph, const R *__restrict__ phi, double alpha,
                          double inv_ebar, double *__restrict__ y) {
    long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const double far_f = -(double)phi[p] + (double)phi[2 * n + p];
    const double far_h = -(double)phi[n + p] + inv_ebar * (double)phi[3 * n + p];
    y[p] = alpha * x[p] + pf[p] + far_f;
    y[n + p] = alpha * x[n + p] + ph[p] + far_h;
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
        k_gather_sources<R><<<grid_for(n, 256), 256, 0, s>>>(x, mp.area, n, mp.sf, mp.sh,
                                                             mp.xp);
        KCHK();
    }
    // fork: the near field (P2P and patch corrections) depends only on the
    // gathered sources and x, and runs beside the far-field chain.  P2P
    // issues at full VALU rate and, started with the chain, holds the SIMDs
    // that P2M waits for; late_p2p puts the memory-bound near correction
    // beside P2M and P2P beside the translations instead.  serial: every
    // kernel on s, one after another.
    const hipStream_t sd = mp.serial ? s : mp.side;
    if (!mp.serial) {
        HIPCHK(hipEventRecord(mp.fork, s));
        HIPCHK(hipStreamWaitEvent(sd, mp.fork, 0));
    }
    auto p2p = [&](int add) {
        ProfScope ps(prof, "p2p", sd);
        const Lists &L = *mp.lists;
        k_p2p<R><<<blocks_ok(L.n_chunks, 64), 64, 0, sd>>>(
            L.ch_lo.p, L.ch_hi.p, L.ch_grp.p, L.grp_tbeg.p, L.grp_tend.p, L.rng_b.p, L.rng_e.p,
            L.ch_rev.p, mp.nd, mp.sf, mp.sh, R(mp.kappa), R(mp.inv_ebar), mp.part, mp.rpart);
        KCHK();
        k_p2p_reduce<<<blocks_ok(L.n_groups, 64), 64, 0, sd>>>(
            L.grp_ptr.p, L.grp_tbeg.p, L.grp_tend.p, mp.part, L.rev_ptr.p, L.rev_idx.p, mp.rpart,
            mp.pf, mp.ph, add);
        KCHK();
    };
    auto near = [&](auto add) {
        ProfScope ps(prof, "near", sd);
        k_near_apply<R, decltype(add)::value><<<grid_for(16 * n, 256), 256, 0, sd>>>(
            n, reinterpret_cast<const typename Pair2<R>::T *>(mp.xp), mp.near->ptr.p,
            mp.near->col.p, mp.delta, mp.pf, mp.ph);
        KCHK();
    };
    if (mp.serial) {
        p2p(0);
        near(std::true_type{});
    } else if (mp.late_p2p) {
        near(std::false_type{});
        // far_field records far.p2m_done after P2M, before it returns
    } else {
        p2p(0);
        near(std::true_type{});
        HIPCHK(hipEventRecord(mp.join, mp.side));
    }
    far_field<R>(*mp.fmm, *mp.tree, *mp.lists, mp.nd64, mp.nd.x, mp.nd.y, mp.nd.z, mp.nd.nx,
                 mp.nd.ny, mp.nd.nz, mp.sf, mp.sh, mp.inv_ebar, n, mp.far, prof, s);
    if (mp.late_p2p && !mp.serial) {
        HIPCHK(hipStreamWaitEvent(sd, mp.far.p2m_done, 0));
        p2p(1);
        HIPCHK(hipEventRecord(mp.join, sd));
    }
    if (!mp.serial) HIPCHK(hipStreamWaitEvent(s, mp.join, 0));
    {
        ProfScope ps(prof, "combine", s);
        k_combine<R><<<grid_for(n, 256), 256, 0, s>>>(n, x, mp.pf, mp.ph, mp.far.phi, mp.alpha,
                                                      mp.inv_ebar, y);
        KCHK();
    }
}

template void apply_operator<double>(const MatvecPlan<double> &, const double *, double *,
                                     Prof *, hipStream_t);
template void apply_operator<float>(const MatvecPlan<float> &, const double *, double *,
                                    Prof *, hipStream_t);

}  // namespace afmpb

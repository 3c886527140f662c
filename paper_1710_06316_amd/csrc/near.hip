// Near set and near-field corrections (Section 2: pairs that are close use
// the patch integrals of Eq. (6), computed once and stored).
//
// Near set: N(p) = {p} U {t : |x_p - x_t|^2 < eta^2 max(rho_p^2, rho_t^2)},
// found with a uniform grid of cell size eta * max(rho); the test itself is
// exact FP64 without fused multiply-add.  For each entry the stored value is
// the patch integral minus the point-rule value (the point rule is what the
// FMM/P2P part of the matvec applies to every pair t != p), so the matvec is
// independent of the octree.
//
// Quadrature over the patch of t: the flat pieces (t, m_tu, c_T) and
// (t, c_T, m_tw) of every incident triangle T = (t, u, w), with T's facet
// normal.  Self patch (t = p): collapsed Gauss product rule with the
// singular vertex at p, 16 x 16 points, facet normal as target normal (so
// the B and C integrands vanish).  Other patches: midpoint subdivision of a
// piece while the target is closer than two diameters to its centroid (at
// most 10 levels), then an 8 x 8 collapsed Gauss rule per piece.
#include "geometry.h"
#include "kernels.h"
#include "near.h"

namespace afmpb {

namespace {

#pragma clang fp contract(off)

// x / 3 rounded to nearest: the product with the rounded reciprocal, then one
// correction by the exact remainder x - 3 q (an FMA).  Equal to the IEEE
// quotient (checked on 4e8 random doubles), at a fraction of a division.
__device__ inline double div3(double x) {
    const double y = 1.0 / 3.0;
    const double q = x * y;
    return fma(fma(-q, 3.0, x), y, q);
}

__device__ inline double dist2(double ax, double ay, double az, double bx, double by, double bz) {
    double dx = ax - bx, dy = ay - by, dz = az - bz;
    return (dx * dx + dy * dy) + dz * dz;
}

__global__ void k_cell_keys(NodeSoA nd, long long n, double lx, double ly, double lz,
                            double inv_cell, long long ny_, long long nz_,
                            unsigned long long *keys, int *idx) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    long long cx = (long long)floor((nd.x[i] - lx) * inv_cell);
    long long cy = (long long)floor((nd.y[i] - ly) * inv_cell);
    long long cz = (long long)floor((nd.z[i] - lz) * inv_cell);
    keys[i] = (unsigned long long)((cx * ny_ + cy) * nz_ + cz);
    idx[i] = (int)i;
}

__device__ inline long long lower_bound_u64(const unsigned long long *a, long long n,
                                            unsigned long long v) {
    long long lo = 0, hi = n;
    while (lo < hi) {
        long long mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

template <bool FILL>
__global__ void k_near(NodeSoA nd, long long n, double lx, double ly, double lz,
                       double inv_cell, long long nx_, long long ny_, long long nz_,
                       const unsigned long long *__restrict__ ckeys, const int *__restrict__ cidx,
                       double eta2, int *cnt, const long long *ptr, int *col, int *err) {
    long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const double px = nd.x[p], py = nd.y[p], pz = nd.z[p], rp = nd.rho2[p];
    long long cx = (long long)floor((px - lx) * inv_cell);
    long long cy = (long long)floor((py - ly) * inv_cell);
    long long cz = (long long)floor((pz - lz) * inv_cell);
    int c = 0;
    long long o = FILL ? ptr[p] : 0;
    for (long long ix = cx - 1; ix <= cx + 1; ++ix) {
        if (ix < 0 || ix >= nx_) continue;
        for (long long iy = cy - 1; iy <= cy + 1; ++iy) {
            if (iy < 0 || iy >= ny_) continue;
            for (long long iz = cz - 1; iz <= cz + 1; ++iz) {
                if (iz < 0 || iz >= nz_) continue;
                unsigned long long key = (unsigned long long)((ix * ny_ + iy) * nz_ + iz);
                long long b = lower_bound_u64(ckeys, n, key);
                for (long long q = b; q < n && ckeys[q] == key; ++q) {
                    int t = cidx[q];
                    bool near;
                    if (t == p) {
                        near = true;
                    } else {
                        double dd = dist2(px, py, pz, nd.x[t], nd.y[t], nd.z[t]);
                        double r2 = rp > nd.rho2[t] ? rp : nd.rho2[t];
                        near = dd < eta2 * r2;
                    }
                    if (near) {
                        if (FILL) {
                            if (o + c < ptr[p + 1]) col[o + c] = t;
                            else atomicOr(err, 1);
                        }
                        ++c;
                    }
                }
            }
        }
    }
    if (!FILL) cnt[p] = c;
    else if (o + c != ptr[p + 1]) atomicOr(err, 1);
}

__global__ void k_sort_rows64(const long long *ptr, int *idx, long long nrows) {
    long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    long long b = ptr[r], e = ptr[r + 1];
    for (long long i = b + 1; i < e; ++i) {
        int v = idx[i];
        long long j = i - 1;
        while (j >= b && idx[j] > v) { idx[j + 1] = idx[j]; --j; }
        idx[j + 1] = v;
    }
}

__global__ void k_count_to_i64(const int *c, long long *o, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = c[i];
}

// ----------------------------- quadrature ----------------------------------

struct Ctx {
    const double *V;           // caller-order coordinates [n][3]
    const int *T;              // [m][3]
    const double *tri_n;       // [m][3]
    const int *inc_ptr, *inc_tri;
    const int *perm;           // Morton position -> caller index
    NodeSoA nd;                // Morton order
    double kappa, inv_ebar;
    // (u, v, weight product) of the collapsed Gauss rules: 64 points of the
    // 8 x 8 rule, then 256 points of the 16 x 16 rule
    const double *rule;
};

constexpr int MAX_DEPTH = 10;

__device__ inline double tri_area(const double *P0, const double *P1, const double *P2) {
    const double e1x = P1[0] - P0[0], e1y = P1[1] - P0[1], e1z = P1[2] - P0[2];
    const double e2x = P2[0] - P0[0], e2y = P2[1] - P0[1], e2z = P2[2] - P0[2];
    const double cx = e1y * e2z - e1z * e2y;
    const double cy = e1z * e2x - e1x * e2z;
    const double cz = e1x * e2y - e1y * e2x;
    return 0.5 * sqrt((cx * cx + cy * cy) + cz * cz);
}

// Vertices of piece `half` of incident triangle k of node ot: (t, m_tu, c_T)
// or (t, c_T, m_tw), and the facet normal.
__device__ inline void piece_root(const Ctx &C, long long ot, long long k, int half, double *R0,
                                  double *R1, double *R2, double &fnx, double &fny, double &fnz) {
    const int *tv = C.T + 3 * k;
    const int i0 = tv[0], i1 = tv[1], i2 = tv[2];
    const int jj = (i0 == ot) ? 0 : ((i1 == ot) ? 1 : 2);
    const int iu = jj == 0 ? i1 : (jj == 1 ? i2 : i0);
    const int iw = jj == 0 ? i2 : (jj == 1 ? i0 : i1);
    const double *vt = C.V + 3 * ot, *pu = C.V + 3ll * iu, *pw = C.V + 3ll * iw;
    const double *a = C.V + 3ll * i0, *b = C.V + 3ll * i1, *c = C.V + 3ll * i2;
    for (int d = 0; d < 3; ++d) {
        const double cen = div3((a[d] + b[d]) + c[d]);
        R0[d] = vt[d];
        R1[d] = half ? cen : (vt[d] + pu[d]) * 0.5;
        R2[d] = half ? (vt[d] + pw[d]) * 0.5 : cen;
    }
    fnx = C.tri_n[3 * k];
    fny = C.tri_n[3 * k + 1];
    fnz = C.tri_n[3 * k + 2];
}

// Sub-triangle c of (P0, P1, P2) under midpoint subdivision, in place.
__device__ inline void to_child(double *P0, double *P1, double *P2, int c) {
    for (int d = 0; d < 3; ++d) {
        const double m01 = (P0[d] + P1[d]) * 0.5;
        const double m12 = (P1[d] + P2[d]) * 0.5;
        const double m20 = (P2[d] + P0[d]) * 0.5;
        double a, b, cc;
        switch (c) {
            case 0: a = P0[d]; b = m01; cc = m20; break;
            case 1: a = m01; b = P1[d]; cc = m12; break;
            case 2: a = m20; b = m12; cc = P2[d]; break;
            default: a = m12; b = m20; cc = m01; break;
        }
        P0[d] = a; P1[d] = b; P2[d] = cc;
    }
}

__device__ inline double wave_add(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One wavefront per near entry (t in N(p)).  The wave walks t's pieces and
// their subdivision trees in a fixed order (the walk is uniform across
// lanes); every step of the loop evaluates one quadrature point per lane, so
// the point kernel is inlined once.  A piece is split while the target is
// closer than two diameters to its centroid (at most MAX_DEPTH levels; the
// path is kept as base-4 digits in one integer and the piece rebuilt from
// its root); every leaf piece gets the 8 x 8 collapsed rule
// y = P0 + u (P1 - P0) + u v (P2 - P1), dS = 2 |tau| u du dv (lane l: point
// l).  The self patch takes the 16 x 16 rule unsplit, lane l evaluating
// points l, l + 64, l + 128, l + 192 in four steps.  Lane sums are added by a
// fixed butterfly at the end.
// Register budget: 4 waves per SIMD (a few spills of loop-invariant values
// cost less than the latency hiding they buy for the FP64 point kernel).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_near_coeffs(Ctx C, long long n, long long nnz, const long long *__restrict__ ptr,
              const int *__restrict__ col, double *__restrict__ delta) {
    const int lane = threadIdx.x & 63;
    const double u8 = C.rule[3 * lane], v8 = C.rule[3 * lane + 1], g8 = C.rule[3 * lane + 2];
    // grid-stride over the entries, so that the launch stays far below the
    // 2^32 work-item limit of one dispatch; the entry index is made visibly
    // wave-uniform so that the walk's addresses and loads stay scalar
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (long long e = (long long)blockIdx.x * 4 + wave; e < nnz;
         e += (long long)gridDim.x * 4) {
        long long lo = 0, hi = n;              // row p: ptr[p] <= e < ptr[p+1]
        while (hi - lo > 1) {
            long long mid = (lo + hi) >> 1;
            if (ptr[mid] <= e) lo = mid; else hi = mid;
        }
        const long long p = lo;
        const double x = C.nd.x[p], y = C.nd.y[p], z = C.nd.z[p];
        const int t = col[e];
        const bool self = t == p;
        double n0x = C.nd.nx[p], n0y = C.nd.ny[p], n0z = C.nd.nz[p];
        const long long ot = C.perm[t];
        double acc_a = 0, acc_b = 0, acc_c = 0, acc_d = 0;
        const int q_end = C.inc_ptr[ot + 1];
        int q = C.inc_ptr[ot], half = 0;
        double R0[3], R1[3], R2[3], fnx = 0, fny = 0, fnz = 0;
        double rarea = 0;                      // area of the current root piece
        if (q < q_end) {
            piece_root(C, ot, C.inc_tri[q], 0, R0, R1, R2, fnx, fny, fnz);
            rarea = tri_area(R0, R1, R2);
        }
        unsigned path = 0;                     // digit k in bits 2k, 2k+1
        int depth = 0, sub = 0;                // sub: self-rule step 0..3
        while (q < q_end) {
            double P0[3], P1[3], P2[3];
            for (int d = 0; d < 3; ++d) { P0[d] = R0[d]; P1[d] = R1[d]; P2[d] = R2[d]; }
            for (int k = 0; k < depth; ++k) to_child(P0, P1, P2, (path >> (2 * k)) & 3);
            if (!self) {
                while (depth < MAX_DEPTH) {    // descend through child 0 while too close
                    const double cx = div3((P0[0] + P1[0]) + P2[0]);
                    const double cy = div3((P0[1] + P1[1]) + P2[1]);
                    const double cz = div3((P0[2] + P1[2]) + P2[2]);
                    double dm = dist2(P0[0], P0[1], P0[2], P1[0], P1[1], P1[2]);
                    const double d12 = dist2(P1[0], P1[1], P1[2], P2[0], P2[1], P2[2]);
                    const double d20 = dist2(P2[0], P2[1], P2[2], P0[0], P0[1], P0[2]);
                    if (d12 > dm) dm = d12;
                    if (d20 > dm) dm = d20;
                    if (!(dist2(x, y, z, cx, cy, cz) < 4.0 * dm)) break;
                    to_child(P0, P1, P2, 0);   // digit 0 adds no bits to the path
                    ++depth;
                }
            }
            double u = u8, v = v8, g = g8;
            if (self) {
                const double *r = C.rule + 3 * (64 + lane + 64 * sub);
                u = r[0]; v = r[1]; g = r[2];
                n0x = fnx; n0y = fny; n0z = fnz;
            }
            {
                // a piece of depth d is a quarter^d of its root (midpoint split)
                const double area = ldexp(rarea, -2 * depth);
                const double w = 2.0 * area * u * g;
                const double yx = P0[0] + u * (P1[0] - P0[0]) + u * v * (P2[0] - P1[0]);
                const double yy = P0[1] + u * (P1[1] - P0[1]) + u * v * (P2[1] - P1[1]);
                const double yz = P0[2] + u * (P1[2] - P0[2]) + u * v * (P2[2] - P1[2]);
                Abcd<double> kk = abcd_point(x - yx, y - yy, z - yz, n0x, n0y, n0z, fnx, fny,
                                             fnz, C.kappa, C.inv_ebar);
                acc_a += w * kk.A;
                acc_b += w * kk.B;
                acc_c += w * kk.C;
                acc_d += w * kk.D;
            }
            // advance: next self-rule step, next leaf of the walk, next piece
            bool next_piece;
            if (self) {
                next_piece = ++sub == 4;
                if (next_piece) sub = 0;
            } else {
                while (depth > 0 && ((path >> (2 * (depth - 1))) & 3) == 3) {
                    path &= ~(3u << (2 * (depth - 1)));
                    --depth;
                }
                next_piece = depth == 0;
                if (!next_piece) path += 1u << (2 * (depth - 1));
            }
            if (next_piece) {
                half ^= 1;
                if (half == 0) ++q;
                if (q < q_end) {
                    piece_root(C, ot, C.inc_tri[q], half, R0, R1, R2, fnx, fny, fnz);
                    rarea = tri_area(R0, R1, R2);
                }
            }
        }
        acc_a = wave_add(acc_a);
        acc_b = wave_add(acc_b);
        acc_c = wave_add(acc_c);
        acc_d = wave_add(acc_d);
        if (lane == 0) {
            if (!self) {   // subtract the point rule applied by the far-field part
                const double at = C.nd.area[t];
                Abcd<double> kp = abcd_point(x - C.nd.x[t], y - C.nd.y[t], z - C.nd.z[t], n0x,
                                             n0y, n0z, C.nd.nx[t], C.nd.ny[t], C.nd.nz[t],
                                             C.kappa, C.inv_ebar);
                acc_a -= at * kp.A;
                acc_b -= at * kp.B;
                acc_c -= at * kp.C;
                acc_d -= at * kp.D;
            } else {       // flat facet: the B and C integrands vanish
                acc_b = 0;
                acc_c = 0;
            }
            delta[4 * e] = acc_a;
            delta[4 * e + 1] = acc_b;
            delta[4 * e + 2] = acc_c;
            delta[4 * e + 3] = acc_d;
        }
    }
}

// grid-stride: 4 nnz passes the 2^32 work-item limit of a dispatch on
// surfaces of ~10M nodes
__global__ void k_round_f32(const double *a, float *b, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

}  // namespace

// Gauss-Legendre nodes and weights on [0,1] (Newton iteration on P_n).
void gauss_legendre01(int nq, double *x, double *w) {
    for (int i = 0; i < nq; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (nq + 0.5));
        double pd = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= nq; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            pd = nq * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / pd;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= nq; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        pd = nq * (z * p1 - p0) / (z * z - 1.0);
        x[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * pd * pd);
    }
}

void build_near(const NodeSoA &nd, long long n, double eta, NearSet &out, hipStream_t s) {
    // grid of cell size eta * max(rho), padded by a relative 1e-9
    std::vector<double> hx(n), hy(n), hz(n), hr(n);
    HIPCHK(hipMemcpyAsync(hr.data(), nd.rho2, n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hx.data(), nd.x, n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hy.data(), nd.y, n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hz.data(), nd.z, n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double rmax2 = 0.0, lo[3] = {1e308, 1e308, 1e308}, hi[3] = {-1e308, -1e308, -1e308};
    for (long long i = 0; i < n; ++i) {
        rmax2 = std::fmax(rmax2, hr[i]);
        const double c[3] = {hx[i], hy[i], hz[i]};
        for (int a = 0; a < 3; ++a) { lo[a] = std::fmin(lo[a], c[a]); hi[a] = std::fmax(hi[a], c[a]); }
    }
    double cell = eta * std::sqrt(rmax2) * (1.0 + 1e-9);
    double ext = std::fmax(hi[0] - lo[0], std::fmax(hi[1] - lo[1], hi[2] - lo[2]));
    if (cell < ext * 1e-6) cell = ext * 1e-6;  // bounds the grid size
    if (cell <= 0) cell = 1.0;
    double inv_cell = 1.0 / cell;
    long long dims[3];
    for (int a = 0; a < 3; ++a) dims[a] = (long long)std::floor((hi[a] - lo[a]) * inv_cell) + 2;
    DBuf<unsigned long long> ck(n), tk(n);
    DBuf<int> ci(n), ti(n);
    k_cell_keys<<<grid_for(n, 256), 256, 0, s>>>(nd, n, lo[0], lo[1], lo[2], inv_cell, dims[1],
                                                 dims[2], ck.p, ci.p);
    KCHK();
    unsigned long long maxkey = (unsigned long long)(dims[0] * dims[1] * dims[2]);
    int bits = 1;
    while (bits < 64 && (maxkey >> bits)) ++bits;
    radix_sort_pairs(ck.p, ci.p, tk.p, ti.p, n, bits, s);
    double eta2 = eta * eta;
    DBuf<int> cnt(n + 1), nerr(1);
    nerr.zero(1, s);
    DBuf<long long> cnt64(n + 1);
    k_near<false><<<grid_for(n, 128), 128, 0, s>>>(nd, n, lo[0], lo[1], lo[2], inv_cell, dims[0],
                                                   dims[1], dims[2], ck.p, ci.p, eta2, cnt.p,
                                                   nullptr, nullptr, nullptr);
    KCHK();
    k_count_to_i64<<<grid_for(n, 256), 256, 0, s>>>(cnt.p, cnt64.p, n);
    KCHK();
    out.ptr.alloc(n + 1);
    exclusive_scan_i64(cnt64.p, out.ptr.p, n, s);
    HIPCHK(hipMemcpyAsync(&out.nnz, out.ptr.p + n, sizeof(long long), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    out.col.alloc(out.nnz);
    k_near<true><<<grid_for(n, 128), 128, 0, s>>>(nd, n, lo[0], lo[1], lo[2], inv_cell, dims[0],
                                                  dims[1], dims[2], ck.p, ci.p, eta2, nullptr,
                                                  out.ptr.p, out.col.p, nerr.p);
    KCHK();
    {
        int herr = 0;
        HIPCHK(hipMemcpyAsync(&herr, nerr.p, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        require(herr == 0, ST_DEVICE, "near-set fill out of range");
    }
    k_sort_rows64<<<grid_for(n, 256), 256, 0, s>>>(out.ptr.p, out.col.p, n);
    KCHK();
    HIPCHK(hipStreamSynchronize(s));
}

void near_coeffs(const NodeSoA &nd, long long n, const double *V, const int *T,
                 const double *tri_n, const int *inc_ptr, const int *inc_tri, const int *perm,
                 double kappa, double ebar, NearSet &out, hipStream_t s) {
    // patch-integral corrections
    Ctx C;
    C.V = V; C.T = T; C.tri_n = tri_n; C.inc_ptr = inc_ptr; C.inc_tri = inc_tri; C.perm = perm;
    C.nd = nd; C.kappa = kappa; C.inv_ebar = 1.0 / ebar;
    double x8[8], w8[8], x16[16], w16[16];
    gauss_legendre01(8, x8, w8);
    gauss_legendre01(16, x16, w16);
    std::vector<double> rule(3 * (64 + 256));
    for (int l = 0; l < 64; ++l) {
        rule[3 * l] = x8[l >> 3];
        rule[3 * l + 1] = x8[l & 7];
        rule[3 * l + 2] = w8[l >> 3] * w8[l & 7];
    }
    for (int l = 0; l < 256; ++l) {
        double *r = &rule[3 * (64 + l)];
        r[0] = x16[l >> 4];
        r[1] = x16[l & 15];
        r[2] = w16[l >> 4] * w16[l & 15];
    }
    out.rule.alloc(rule.size());
    HIPCHK(hipMemcpyAsync(out.rule.p, rule.data(), rule.size() * sizeof(double),
                          hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));      // the host table must outlive the copy
    C.rule = out.rule.p;
    out.delta.alloc(4 * out.nnz);
    // one wave per entry, at most 2^22 blocks of 4 waves (the kernel strides)
    const long long nblk = std::min<long long>((out.nnz + 3) / 4, 1ll << 22);
    k_near_coeffs<<<(unsigned)std::max(nblk, 1ll), 256, 0, s>>>(C, n, out.nnz, out.ptr.p,
                                                               out.col.p, out.delta.p);
    KCHK();
    out.delta32.alloc(4 * out.nnz);
    k_round_f32<<<(unsigned)std::min<long long>((4 * out.nnz + 255) / 256, 1ll << 20), 256, 0, s>>>(
        out.delta.p, out.delta32.p, 4 * out.nnz);
    KCHK();
}

}  // namespace afmpb

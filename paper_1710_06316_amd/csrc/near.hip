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

struct QuadRules {
    double x8[8], w8[8], x16[16], w16[16];
};

struct Ctx {
    const double *V;           // caller-order coordinates [n][3]
    const int *T;              // [m][3]
    const double *tri_n;       // [m][3]
    const int *inc_ptr, *inc_tri;
    const int *perm;           // Morton position -> caller index
    NodeSoA nd;                // Morton order
    double kappa, inv_ebar;
    QuadRules q;
};

struct Acc {
    double a, b, c, d;
};

__device__ inline void child_of(const double *P0, const double *P1, const double *P2, int c,
                                double *Q0, double *Q1, double *Q2) {
    double m01[3], m12[3], m20[3];
    for (int d = 0; d < 3; ++d) {
        m01[d] = (P0[d] + P1[d]) * 0.5;
        m12[d] = (P1[d] + P2[d]) * 0.5;
        m20[d] = (P2[d] + P0[d]) * 0.5;
    }
    const double *a, *b, *cc;
    switch (c) {
        case 0: a = P0; b = m01; cc = m20; break;
        case 1: a = m01; b = P1; cc = m12; break;
        case 2: a = m20; b = m12; cc = P2; break;
        default: a = m12; b = m20; cc = m01; break;
    }
    for (int d = 0; d < 3; ++d) { Q0[d] = a[d]; Q1[d] = b[d]; Q2[d] = cc[d]; }
}

constexpr int MAX_DEPTH = 10;

// One wavefront per near entry (t in N(p)): the wave walks t's pieces and
// their subdivision tree together (the walk is uniform across lanes), and
// lane l evaluates point (l / 8, l % 8) of the 8 x 8 collapsed rule of every
// leaf piece (self patch: points l, l+64, l+128, l+192 of the 16 x 16 rule).
// Lane sums are added by a fixed butterfly at the end.
struct LanePts {
    double u8, v8, g8;          // node and weight product of this lane's 8 x 8 point
    double u16[4], v16[4], g16[4];
};

__device__ inline void piece_lane(const Ctx &C, double x, double y0, double z, double n0x,
                                  double n0y, double n0z, const double *P0, const double *P1,
                                  const double *P2, double fnx, double fny, double fnz,
                                  int npts, const double *uu, const double *vv, const double *gg,
                                  bool self, Acc &acc) {
    double e1[3] = {P1[0] - P0[0], P1[1] - P0[1], P1[2] - P0[2]};
    double e2[3] = {P2[0] - P0[0], P2[1] - P0[1], P2[2] - P0[2]};
    double cx = e1[1] * e2[2] - e1[2] * e2[1];
    double cy = e1[2] * e2[0] - e1[0] * e2[2];
    double cz = e1[0] * e2[1] - e1[1] * e2[0];
    double area = 0.5 * sqrt((cx * cx + cy * cy) + cz * cz);
    for (int s = 0; s < npts; ++s) {
        const double u = uu[s], v = vv[s];
        const double w = 2.0 * area * u * gg[s];
        double pyy[3];
        for (int d = 0; d < 3; ++d)
            pyy[d] = P0[d] + u * (P1[d] - P0[d]) + u * v * (P2[d] - P1[d]);
        const double rx = x - pyy[0], ry = y0 - pyy[1], rz = z - pyy[2];
        if (self) {
            Abcd<double> k = abcd_point(rx, ry, rz, fnx, fny, fnz, fnx, fny, fnz, C.kappa,
                                        C.inv_ebar);
            acc.a += w * k.A;
            acc.d += w * k.D;
        } else {
            Abcd<double> k = abcd_point(rx, ry, rz, n0x, n0y, n0z, fnx, fny, fnz, C.kappa,
                                        C.inv_ebar);
            acc.a += w * k.A;
            acc.b += w * k.B;
            acc.c += w * k.C;
            acc.d += w * k.D;
        }
    }
}

// Adaptive subdivision of one piece, depth first, with the path kept as
// base-4 digits and the current sub-triangle rebuilt from the root; a piece
// is split while the target is closer than two diameters to its centroid
// (at most MAX_DEPTH levels), and every leaf gets the 8 x 8 collapsed rule
// y = P0 + u (P1 - P0) + u v (P2 - P1), dS = 2 |tau| u du dv (collapse at P0).
__device__ void adapt_lane(const Ctx &C, double x, double y, double z, double n0x, double n0y,
                           double n0z, const double *R0, const double *R1, const double *R2,
                           double fnx, double fny, double fnz, const LanePts &L, Acc &acc) {
    int digit[MAX_DEPTH + 1];
    int depth = 0;
    while (true) {
        double P0[3], P1[3], P2[3];
        for (int d = 0; d < 3; ++d) { P0[d] = R0[d]; P1[d] = R1[d]; P2[d] = R2[d]; }
        for (int k = 0; k < depth; ++k) {
            double Q0[3], Q1[3], Q2[3];
            child_of(P0, P1, P2, digit[k], Q0, Q1, Q2);
            for (int d = 0; d < 3; ++d) { P0[d] = Q0[d]; P1[d] = Q1[d]; P2[d] = Q2[d]; }
        }
        double cx = ((P0[0] + P1[0]) + P2[0]) / 3.0;
        double cy = ((P0[1] + P1[1]) + P2[1]) / 3.0;
        double cz = ((P0[2] + P1[2]) + P2[2]) / 3.0;
        double dm = dist2(P0[0], P0[1], P0[2], P1[0], P1[1], P1[2]);
        double d12 = dist2(P1[0], P1[1], P1[2], P2[0], P2[1], P2[2]);
        double d20 = dist2(P2[0], P2[1], P2[2], P0[0], P0[1], P0[2]);
        if (d12 > dm) dm = d12;
        if (d20 > dm) dm = d20;
        if (depth < MAX_DEPTH && dist2(x, y, z, cx, cy, cz) < 4.0 * dm) {
            digit[depth++] = 0;
            continue;
        }
        piece_lane(C, x, y, z, n0x, n0y, n0z, P0, P1, P2, fnx, fny, fnz, 1, &L.u8, &L.v8, &L.g8,
                   false, acc);
        while (depth > 0 && digit[depth - 1] == 3) --depth;
        if (depth == 0) break;
        ++digit[depth - 1];
    }
}

__device__ inline double wave_add(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ void __launch_bounds__(256) k_near_coeffs(Ctx C, long long n, long long nnz,
                                                     const long long *__restrict__ ptr,
                                                     const int *__restrict__ col,
                                                     double *__restrict__ delta) {
    const int lane = threadIdx.x & 63;
    LanePts L;
    {
        const int i = lane >> 3, j = lane & 7;
        L.u8 = C.q.x8[i];
        L.v8 = C.q.x8[j];
        L.g8 = C.q.w8[i] * C.q.w8[j];
        for (int s = 0; s < 4; ++s) {
            const int idx = lane + 64 * s, i2 = idx >> 4, j2 = idx & 15;
            L.u16[s] = C.q.x16[i2];
            L.v16[s] = C.q.x16[j2];
            L.g16[s] = C.q.w16[i2] * C.q.w16[j2];
        }
    }
    // grid-stride over the entries (wave-uniform), so that the launch stays
    // far below the 2^32 work-item limit of one dispatch
    for (long long e = (long long)blockIdx.x * 4 + (threadIdx.x >> 6); e < nnz;
         e += (long long)gridDim.x * 4) {
    long long lo = 0, hi = n;              // row p: ptr[p] <= e < ptr[p+1]
    while (hi - lo > 1) {
        long long mid = (lo + hi) >> 1;
        if (ptr[mid] <= e) lo = mid; else hi = mid;
    }
    const long long p = lo;
    const double x = C.nd.x[p], y = C.nd.y[p], z = C.nd.z[p];
    const double n0x = C.nd.nx[p], n0y = C.nd.ny[p], n0z = C.nd.nz[p];
    const int t = col[e];
    const long long ot = C.perm[t];
    const double *vt = C.V + 3 * ot;
    Acc acc{0, 0, 0, 0};
    for (int q = C.inc_ptr[ot]; q < C.inc_ptr[ot + 1]; ++q) {
        long long k = C.inc_tri[q];
        const int *tv = C.T + 3 * k;
        int jj = (tv[0] == ot) ? 0 : ((tv[1] == ot) ? 1 : 2);
        const double *pu = C.V + 3ll * tv[(jj + 1) % 3];
        const double *pw = C.V + 3ll * tv[(jj + 2) % 3];
        const double *a = C.V + 3ll * tv[0], *b = C.V + 3ll * tv[1], *c = C.V + 3ll * tv[2];
        double cen[3], mu[3], mw[3];
        for (int d = 0; d < 3; ++d) {
            cen[d] = ((a[d] + b[d]) + c[d]) / 3.0;
            mu[d] = (vt[d] + pu[d]) * 0.5;
            mw[d] = (vt[d] + pw[d]) * 0.5;
        }
        double fnx = C.tri_n[3 * k], fny = C.tri_n[3 * k + 1], fnz = C.tri_n[3 * k + 2];
        if (t == p) {
            piece_lane(C, x, y, z, n0x, n0y, n0z, vt, mu, cen, fnx, fny, fnz, 4, L.u16, L.v16,
                       L.g16, true, acc);
            piece_lane(C, x, y, z, n0x, n0y, n0z, vt, cen, mw, fnx, fny, fnz, 4, L.u16, L.v16,
                       L.g16, true, acc);
        } else {
            adapt_lane(C, x, y, z, n0x, n0y, n0z, vt, mu, cen, fnx, fny, fnz, L, acc);
            adapt_lane(C, x, y, z, n0x, n0y, n0z, vt, cen, mw, fnx, fny, fnz, L, acc);
        }
    }
    acc.a = wave_add(acc.a);
    acc.b = wave_add(acc.b);
    acc.c = wave_add(acc.c);
    acc.d = wave_add(acc.d);
    if (lane == 0) {
        if (t != p) {   // subtract the point rule applied by the far-field part
            double at = C.nd.area[t];
            Abcd<double> kp = abcd_point(x - C.nd.x[t], y - C.nd.y[t], z - C.nd.z[t], n0x, n0y,
                                         n0z, C.nd.nx[t], C.nd.ny[t], C.nd.nz[t], C.kappa,
                                         C.inv_ebar);
            acc.a -= at * kp.A;
            acc.b -= at * kp.B;
            acc.c -= at * kp.C;
            acc.d -= at * kp.D;
        }
        delta[4 * e] = acc.a;
        delta[4 * e + 1] = acc.b;
        delta[4 * e + 2] = acc.c;
        delta[4 * e + 3] = acc.d;
    }
    }
}

__global__ void k_round_f32(const double *a, float *b, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
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

void build_near(const NodeSoA &nd, long long n, double eta, const double *V, const int *T,
                const double *tri_n, const int *inc_ptr, const int *inc_tri, const int *perm,
                double kappa, double ebar, NearSet &out, hipStream_t s) {
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
    // patch-integral corrections
    Ctx C;
    C.V = V; C.T = T; C.tri_n = tri_n; C.inc_ptr = inc_ptr; C.inc_tri = inc_tri; C.perm = perm;
    C.nd = nd; C.kappa = kappa; C.inv_ebar = 1.0 / ebar;
    gauss_legendre01(8, C.q.x8, C.q.w8);
    gauss_legendre01(16, C.q.x16, C.q.w16);
    out.delta.alloc(4 * out.nnz);
    // one wave per entry, at most 2^22 blocks of 4 waves (the kernel strides)
    const long long nblk = std::min<long long>((out.nnz + 3) / 4, 1ll << 22);
    k_near_coeffs<<<(unsigned)std::max(nblk, 1ll), 256, 0, s>>>(C, n, out.nnz, out.ptr.p,
                                                               out.col.p, out.delta.p);
    KCHK();
    out.delta32.alloc(4 * out.nnz);
    k_round_f32<<<grid_for(4 * out.nnz, 256), 256, 0, s>>>(out.delta.p, out.delta32.p, 4 * out.nnz);
    KCHK();
    HIPCHK(hipStreamSynchronize(s));
}

}  // namespace afmpb

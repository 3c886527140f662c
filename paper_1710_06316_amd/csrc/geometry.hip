// Patch geometry of the node-patch scheme (Section 2, Figure 1) and Morton
// keys.  Everything here is FP64 with fused multiply-add disabled so that the
// near-set test and the tree quantisation are reproducible bit for bit.
#include "geometry.h"

namespace afmpb {

namespace {

#pragma clang fp contract(off)

__global__ void k_tri_geometry(const double *__restrict__ V, const int *__restrict__ T,
                               long long m, double *__restrict__ area,
                               double *__restrict__ tn) {
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const double *a = V + 3ll * T[3 * k], *b = V + 3ll * T[3 * k + 1], *c = V + 3ll * T[3 * k + 2];
    double e1x = b[0] - a[0], e1y = b[1] - a[1], e1z = b[2] - a[2];
    double e2x = c[0] - a[0], e2y = c[1] - a[1], e2z = c[2] - a[2];
    double cx = e1y * e2z - e1z * e2y;
    double cy = e1z * e2x - e1x * e2z;
    double cz = e1x * e2y - e1y * e2x;
    double len = sqrt((cx * cx + cy * cy) + cz * cz);
    area[k] = 0.5 * len;
    tn[3 * k] = cx / len;
    tn[3 * k + 1] = cy / len;
    tn[3 * k + 2] = cz / len;
}

__global__ void k_count_incidence(const int *__restrict__ T, long long m, int *cnt) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * m) return;
    atomicAdd(&cnt[T[i]], 1);
}

__global__ void k_fill_incidence(const int *__restrict__ T, long long m,
                                 const int *__restrict__ ptr, int *cursor, int *inc, int *err) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * m) return;
    int v = T[i];
    int slot = atomicAdd(&cursor[v], 1);
    if (ptr[v] + slot >= ptr[v + 1]) { atomicOr(err, 1); return; }
    inc[ptr[v] + slot] = (int)(i / 3);
}

__device__ inline double d2(double ax, double ay, double az, double bx, double by, double bz) {
    double dx = ax - bx, dy = ay - by, dz = az - bz;
    return (dx * dx + dy * dy) + dz * dz;
}

// Per node (caller order), incident triangles in ascending order: patch area
// (a third of each triangle), area-weighted normal, squared patch radius.
__global__ void k_node_geometry(const double *__restrict__ V, const int *__restrict__ T,
                                const double *__restrict__ ta, const double *__restrict__ tn,
                                const int *__restrict__ ptr, const int *__restrict__ inc,
                                long long n, double *__restrict__ area,
                                double *__restrict__ nrm, double *__restrict__ rho2) {
    long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    double A = 0.0, nx = 0.0, ny = 0.0, nz = 0.0, r2 = 0.0;
    const double px = V[3 * v], py = V[3 * v + 1], pz = V[3 * v + 2];
    for (int q = ptr[v]; q < ptr[v + 1]; ++q) {
        long long k = inc[q];
        double a = ta[k];
        A += a / 3.0;
        nx += a * tn[3 * k];
        ny += a * tn[3 * k + 1];
        nz += a * tn[3 * k + 2];
        const int i0 = T[3 * k], i1 = T[3 * k + 1], i2 = T[3 * k + 2];
        const int j = (i0 == v) ? 0 : ((i1 == v) ? 1 : 2);
        for (int jj = 1; jj <= 2; ++jj) {
            long long u = T[3 * k + (j + jj) % 3];
            double mx = (px + V[3 * u]) * 0.5, my = (py + V[3 * u + 1]) * 0.5,
                   mz = (pz + V[3 * u + 2]) * 0.5;
            double dd = d2(mx, my, mz, px, py, pz);
            if (dd > r2) r2 = dd;
        }
        double cx = ((V[3ll * i0] + V[3ll * i1]) + V[3ll * i2]) / 3.0;
        double cy = ((V[3ll * i0 + 1] + V[3ll * i1 + 1]) + V[3ll * i2 + 1]) / 3.0;
        double cz = ((V[3ll * i0 + 2] + V[3ll * i1 + 2]) + V[3ll * i2 + 2]) / 3.0;
        double dd = d2(cx, cy, cz, px, py, pz);
        if (dd > r2) r2 = dd;
    }
    double l = sqrt((nx * nx + ny * ny) + nz * nz);
    area[v] = A;
    nrm[3 * v] = nx / l;
    nrm[3 * v + 1] = ny / l;
    nrm[3 * v + 2] = nz / l;
    rho2[v] = r2;
}

// Per-block min/max of each coordinate; partial[blk][0..5] = min xyz, max xyz.
__global__ void k_bbox_partial(const double *__restrict__ V, long long n, double *partial) {
    __shared__ double sm[6][256];
    double mn[3] = {1e308, 1e308, 1e308}, mx[3] = {-1e308, -1e308, -1e308};
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        for (int a = 0; a < 3; ++a) {
            double x = V[3 * i + a];
            mn[a] = fmin(mn[a], x);
            mx[a] = fmax(mx[a], x);
        }
    }
    for (int a = 0; a < 3; ++a) { sm[a][threadIdx.x] = mn[a]; sm[3 + a][threadIdx.x] = mx[a]; }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            for (int a = 0; a < 3; ++a) {
                sm[a][threadIdx.x] = fmin(sm[a][threadIdx.x], sm[a][threadIdx.x + s]);
                sm[3 + a][threadIdx.x] = fmax(sm[3 + a][threadIdx.x], sm[3 + a][threadIdx.x + s]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) partial[6 * blockIdx.x + threadIdx.x] = sm[threadIdx.x][0];
}

// 21-bit quantisation per axis (one rounded subtraction, one rounded
// multiplication, floor, clamp) and bit interleaving x -> 3b, y -> 3b+1,
// z -> 3b+2.
__global__ void k_morton(const double *__restrict__ V, long long n, double lx, double ly,
                         double lz, double scale, unsigned long long *keys, int *idx) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double lo[3] = {lx, ly, lz};
    unsigned long long key = 0;
    for (int a = 0; a < 3; ++a) {
        double d = V[3 * i + a] - lo[a];
        double q = floor(d * scale);
        if (q > 2097151.0) q = 2097151.0;
        if (q < 0.0) q = 0.0;          // (a point below a widened box's rounded corner)
        unsigned long long u = (unsigned long long)q;
        for (int b = 0; b < 21; ++b) key |= ((u >> b) & 1ull) << (3 * b + a);
    }
    keys[i] = key;
    idx[i] = (int)i;
}

__global__ void k_gather_nodes(const double *__restrict__ V, const double *__restrict__ nrm,
                               const double *__restrict__ area, const double *__restrict__ rho2,
                               const int *__restrict__ perm, long long n, NodeSoA out) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    long long o = perm[i];
    out.x[i] = V[3 * o];
    out.y[i] = V[3 * o + 1];
    out.z[i] = V[3 * o + 2];
    out.nx[i] = nrm[3 * o];
    out.ny[i] = nrm[3 * o + 1];
    out.nz[i] = nrm[3 * o + 2];
    out.area[i] = area[o];
    out.rho2[i] = rho2[o];
}

}  // namespace

void compute_geometry(const double *V, const int *T, long long n, long long m,
                      double *tri_area, double *tri_n, int *inc_ptr, int *inc_tri,
                      double *area, double *nrm, double *rho2, hipStream_t s) {
    DBuf<int> cnt(n + 1), cursor(n + 1), err(1);
    err.zero(1, s);
    cnt.zero(n + 1, s);
    cursor.zero(n + 1, s);
    k_tri_geometry<<<grid_for(m, 256), 256, 0, s>>>(V, T, m, tri_area, tri_n);
    KCHK();
    k_count_incidence<<<grid_for(3 * m, 256), 256, 0, s>>>(T, m, cnt.p);
    KCHK();
    exclusive_scan_i32(cnt.p, inc_ptr, n, s);
    k_fill_incidence<<<grid_for(3 * m, 256), 256, 0, s>>>(T, m, inc_ptr, cursor.p, inc_tri, err.p);
    KCHK();
    sort_rows_i32(inc_ptr, inc_tri, n, s);
    k_node_geometry<<<grid_for(n, 256), 256, 0, s>>>(V, T, tri_area, tri_n, inc_ptr, inc_tri,
                                                      n, area, nrm, rho2);
    KCHK();
    int herr = 0;
    HIPCHK(hipMemcpyAsync(&herr, err.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    require(herr == 0, ST_DEVICE, "incidence fill out of range");
}

void morton_sort(const double *V, long long n, unsigned long long *keys, int *perm,
                 double lo_out[3], double *scale_out, hipStream_t s, bool centre_third) {
    int nblk = 256;
    DBuf<double> part(6 * nblk);
    k_bbox_partial<<<nblk, 256, 0, s>>>(V, n, part.p);
    KCHK();
    std::vector<double> hp(6 * nblk);
    part.download(hp.data(), 6 * nblk, s);
    HIPCHK(hipStreamSynchronize(s));
    double lo[3] = {1e308, 1e308, 1e308}, hi[3] = {-1e308, -1e308, -1e308};
    for (int b = 0; b < nblk; ++b)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::fmin(lo[a], hp[6 * b + a]);
            hi[a] = std::fmax(hi[a], hp[6 * b + 3 + a]);
        }
    double S = 0.0;
    for (int a = 0; a < 3; ++a) S = std::fmax(S, hi[a] - lo[a]);
    if (S == 0.0) S = 1.0;
    if (centre_third) {
        // root of side 1.5 S with the centre of the points' box at 1/3 of
        // it on every axis (binary 0.0101...: a third of a side away from
        // the faces of the boxes of every level)
        // (the corner rounded from the centre may lie above the lowest point
        // by an ulp: never above it)
        for (int a = 0; a < 3; ++a) lo[a] = std::fmin(lo[a], 0.5 * (lo[a] + hi[a]) - 0.5 * S);
        S *= 1.5;
    }
    double scale = 2097152.0 / S;
    for (int a = 0; a < 3; ++a) lo_out[a] = lo[a];
    *scale_out = scale;
    k_morton<<<grid_for(n, 256), 256, 0, s>>>(V, n, lo[0], lo[1], lo[2], scale, keys, perm);
    KCHK();
    DBuf<unsigned long long> tk(n);
    DBuf<int> tv(n);
    radix_sort_pairs(keys, perm, tk.p, tv.p, n, 63, s);
}

void gather_nodes(const double *V, const double *nrm, const double *area, const double *rho2,
                  const int *perm, long long n, const NodeSoA &out, hipStream_t s) {
    k_gather_nodes<<<grid_for(n, 256), 256, 0, s>>>(V, nrm, area, rho2, perm, n, out);
    KCHK();
}

}  // namespace afmpb

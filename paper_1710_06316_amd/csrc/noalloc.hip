// Polar energy without any device allocation: the reaction potential of the
// interior Green representation at every atom, phi_reac(r_k) = sum_t a_t
// [ebar h_t G(r_k, r_t) - f_t dG(r_k, r_t)/dn_t], and E = 1/2 sum_k q_k
// phi_reac(r_k) in kcal/mol, for callers that cannot allocate (graph
// capture, serving loops).  The only scratch is one partial sum per block of
// 256 atoms, kept in a fixed device array that every call on a GPU shares.
#include <mutex>

#include "ctx.h"
#include "kernels.h"

namespace afmpb {

// One FP64 partial per block of NOALLOC_BLOCK atoms; a GPU holds this array
// (128 KiB) until the process ends.
constexpr int NOALLOC_BLOCK = 256;
constexpr long long NOALLOC_PARTIALS = 16384;
constexpr long long NOALLOC_MAX_ATOMS = NOALLOC_PARTIALS * NOALLOC_BLOCK;

static __device__ __align__(256) double scratch[NOALLOC_PARTIALS];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[MAX_DEVICES] = {};

// Partial of block b: sum over its atoms k of q_k phi_reac(r_k).  Nodes are
// read in the caller's order (coordinates, unit normals, patch areas and
// x = [f; h]), staged 256 at a time in LDS.
__global__ void __launch_bounds__(NOALLOC_BLOCK)
k_energy_partial(const double *__restrict__ V, const double *__restrict__ nrm,
                 const double *__restrict__ area, const double *__restrict__ x, long long n,
                 const double *__restrict__ ax, const double *__restrict__ q, long long na,
                 double ebar, double *__restrict__ part) {
    __shared__ double S[8][NOALLOC_BLOCK];
    __shared__ double ws[NOALLOC_BLOCK / 64];
    const long long k = (long long)blockIdx.x * NOALLOC_BLOCK + threadIdx.x;
    const bool act = k < na;
    const double px = act ? ax[3 * k] : 0.0, py = act ? ax[3 * k + 1] : 0.0,
                 pz = act ? ax[3 * k + 2] : 0.0;
    double s = 0.0;
    for (long long t0 = 0; t0 < n; t0 += NOALLOC_BLOCK) {
        const long long t = t0 + threadIdx.x;
        __syncthreads();
        if (t < n) {
            S[0][threadIdx.x] = V[3 * t];
            S[1][threadIdx.x] = V[3 * t + 1];
            S[2][threadIdx.x] = V[3 * t + 2];
            S[3][threadIdx.x] = nrm[3 * t];
            S[4][threadIdx.x] = nrm[3 * t + 1];
            S[5][threadIdx.x] = nrm[3 * t + 2];
            S[6][threadIdx.x] = area[t] * x[t];          // a_t f_t
            S[7][threadIdx.x] = area[t] * x[n + t];      // a_t h_t
        }
        __syncthreads();
        const int cnt = (int)min((long long)NOALLOC_BLOCK, n - t0);
        if (act)
            for (int j = 0; j < cnt; ++j) {
                const double rx = px - S[0][j], ry = py - S[1][j], rz = pz - S[2][j];
                const double r2 = (rx * rx + ry * ry) + rz * rz;
                const double ir = 1.0 / sqrt(r2);
                const double Rn = (rx * S[3][j] + ry * S[4][j]) + rz * S[5][j];
                s += ebar * S[7][j] * ir - S[6][j] * Rn * ir * ir * ir;
            }
    }
    double v = act ? q[k] * s * INV_4PI : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < NOALLOC_BLOCK / 64; ++w) t += ws[w];
        part[blockIdx.x] = t;
    }
}

// E = 1/2 (sum of the nblk partials, in block order) * unit factor.
__global__ void __launch_bounds__(64) k_energy_final(const double *__restrict__ part, int nblk,
                                                     double half_unit, double *__restrict__ out) {
    if (threadIdx.x != 0) return;
    double t = 0.0;
    for (int b = 0; b < nblk; ++b) t += part[b];
    *out = half_unit * t;
}

}  // namespace

// Device address of `scratch` on the current device, looked up once per
// device (each GPU holds its own copy of the array at its own address).
double *noalloc_scratch(int device) {
    require(device >= 0 && device < MAX_DEVICES, ST_INVALID, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        require(p != nullptr, ST_DEVICE, "scratch symbol has no device address");
        g_scratch_ptr[device] = static_cast<double *>(p);
    }
    return g_scratch_ptr[device];
}

void energy_noalloc(afmpb_ctx *c, const double *x_dev, double *energy_dev) {
    require(c->na <= NOALLOC_MAX_ATOMS, ST_INVALID,
            "afmpb_energy_dev_noalloc: more atoms than its static scratch holds (4,194,304)");
    require(c->noalloc_part != nullptr, ST_STATE, "static scratch not resolved");
    const long long nblk = c->na > 0 ? (c->na + NOALLOC_BLOCK - 1) / NOALLOC_BLOCK : 0;
    if (nblk > 0) {
        k_energy_partial<<<(unsigned)nblk, NOALLOC_BLOCK, 0, c->stream>>>(
            c->V.p, c->nrm_c.p, c->area_c.p, x_dev, c->n, c->ax.p, c->aq.p, c->na, c->ebar,
            c->noalloc_part);
        KCHK();
    }
    k_energy_final<<<1, 64, 0, c->stream>>>(c->noalloc_part, (int)nblk, 0.5 * unit_scale(),
                                             energy_dev);
    KCHK();
}

}  // namespace afmpb

// Restarted GMRES held on the GPU (Section 3.4; stopping rule Eq. 7).
//
// One Arnoldi step j: w = M v_j (the matvec of Eq. 5), two block Gram-Schmidt
// passes h = V^T w, w -= V h over v_0..v_j, ||w||, the Givens rotations of
// the Hessenberg column and of the right-hand side g, the residual estimate
// |g_{j+1}| against the tolerance, and v_{j+1} = w / ||w||.  Every kernel
// reads j and the convergence flag from device memory, so the whole step is
// one captured graph, replayed for every j; a step launched after the cycle
// has ended changes nothing.  The host issues step j+1 before it reads the
// status of step j, so the GPU never waits for the host within a cycle (one
// extra matvec per cycle is the price).  Reductions add their partial sums
// in a fixed order: results are reproducible run to run.
#include <cmath>

#include "ctx.h"
#include "gmres.h"

namespace afmpb {

namespace {

constexpr int GB = 256;                  // threads per block
constexpr int GCHUNK = GB * 16;          // vector elements per reduction block
constexpr int VG = 8;                    // basis vectors per projection block

__device__ inline double gblock_sum(double v) {
    __shared__ double ws[GB / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) ws[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < GB / 64; ++w) t += ws[w];
    __syncthreads();
    return t;
}

// part[jv][blk] = <V[jv], w> over chunk blk, for jv <= j; block (blk, group
// of VG vectors); w's chunk is held in registers across the group
__global__ void __launch_bounds__(GB) k_proj_partial(const double *__restrict__ V, long long len,
                                                     const double *__restrict__ w, int nblk,
                                                     const GmresState *__restrict__ st,
                                                     double *__restrict__ part) {
    if (st->done) return;
    const int j = st->j;
    const int jv0 = blockIdx.y * VG;
    if (jv0 > j) return;
    const long long base = (long long)blockIdx.x * GCHUNK;
    double wr[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const long long k = base + (long long)i * GB + threadIdx.x;
        wr[i] = k < len ? w[k] : 0.0;
    }
    for (int q = 0; q < VG; ++q) {
        const int jv = jv0 + q;
        if (jv > j) break;                            // uniform
        const double *v = V + (long long)jv * len;
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const long long k = base + (long long)i * GB + threadIdx.x;
            if (k < len) s += v[k] * wr[i];
        }
        s = gblock_sum(s);
        if (threadIdx.x == 0) part[(long long)jv * nblk + blockIdx.x] = s;
    }
}

// out[jv] = sum of the partials of vector jv in block order (jv <= j)
__global__ void __launch_bounds__(GB) k_proj_final(const double *__restrict__ part, int nblk,
                                                   const GmresState *__restrict__ st,
                                                   double *__restrict__ out) {
    if (st->done) return;
    const int jv = blockIdx.x;
    if (jv > st->j) return;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += GB) s += part[(long long)jv * nblk + b];
    s = gblock_sum(s);
    if (threadIdx.x == 0) out[jv] = s;
}

// w -= V[0..j] c
__global__ void k_proj_update(const double *__restrict__ V, long long len,
                              const GmresState *__restrict__ st, const double *__restrict__ c,
                              double *__restrict__ w) {
    if (st->done) return;
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= len) return;
    const int j = st->j;
    double s = 0.0;
    for (int jv = 0; jv <= j; ++jv) s += V[(long long)jv * len + k] * c[jv];
    w[k] += -1.0 * s;
}

// part[blk] = <a, a> over chunk blk (skipped once the cycle is done when
// `guard`)
__global__ void __launch_bounds__(GB) k_norm_partial(const double *__restrict__ a, long long len,
                                                     const GmresState *__restrict__ st, int guard,
                                                     double *__restrict__ part) {
    if (guard && st->done) return;
    const long long base = (long long)blockIdx.x * GCHUNK;
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const long long k = base + (long long)i * GB + threadIdx.x;
        if (k < len) s += a[k] * a[k];
    }
    s = gblock_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(GB) k_norm_final(const double *__restrict__ part, int nblk,
                                                   const GmresState *__restrict__ st, int guard,
                                                   double *__restrict__ out) {
    if (guard && st->done) return;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += GB) s += part[b];
    s = gblock_sum(s);
    if (threadIdx.x == 0) *out = s;
}

// Hessenberg column j from the two projections and ||w||, the earlier
// rotations applied to it, a new rotation, g rotated, the estimate |g_{j+1}|
// tested against the tolerance.
__global__ void k_givens(GmresState *__restrict__ st, double *__restrict__ H,
                         double *__restrict__ cs, double *__restrict__ sn, double *__restrict__ g,
                         const double *__restrict__ h1, const double *__restrict__ h2,
                         const double *__restrict__ hn2, int m) {
    if (threadIdx.x != 0) return;
    if (st->done) {
        st->active = 0;
        return;
    }
    const int j = st->j;
    double *Hc = H + (long long)j * (m + 1);
    for (int i = 0; i <= j; ++i) Hc[i] = h1[i] + h2[i];
    const double hn = sqrt(*hn2);
    if (!isfinite(hn)) st->pad[0] = 1;            // non-finite Arnoldi vector
    for (int i = 0; i < j; ++i) {
        const double a = Hc[i], b = Hc[i + 1];
        Hc[i] = cs[i] * a + sn[i] * b;
        Hc[i + 1] = -sn[i] * a + cs[i] * b;
    }
    Hc[j + 1] = hn;
    const double den = hypot(Hc[j], hn);
    cs[j] = Hc[j] / den;
    sn[j] = hn / den;
    Hc[j] = den;
    Hc[j + 1] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    st->est = fabs(g[j + 1]);
    st->hn = hn;
    st->j = j + 1;
    st->steps += 1;
    st->active = 1;
    const bool conv = st->est <= st->tol || hn == 0.0;
    st->converged = conv ? 1 : 0;
    st->done = (conv || j + 1 == m) ? 1 : 0;
    st->inv = hn != 0.0 ? 1.0 / hn : 0.0;
}

// v_{j+1} = w / ||w|| (and the next matvec input), unless the cycle ended
__global__ void k_next_vector(const double *__restrict__ w, long long len,
                              const GmresState *__restrict__ st, double *__restrict__ V,
                              double *__restrict__ xa) {
    if (!st->active || st->done) return;
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= len) return;
    const double v = st->inv * w[k];
    V[(long long)st->j * len + k] = v;
    xa[k] = v;
}

// run tolerance rel ||b|| + abs; beta holds ||b|| for the host
__global__ void k_set_tol(GmresState *st, const double *nrm2, double rel, double abs_tol) {
    if (threadIdx.x != 0) return;
    const double nb = sqrt(*nrm2);
    st->tol = rel * nb + abs_tol;
    st->beta = nb;
    st->steps = 0;
    st->done = 1;
    st->converged = 0;
    st->j = 0;
    st->active = 0;
    st->pad[0] = 0;
    st->est = nb;
}

// start of a cycle from r0 (in V[0]) with squared norm *nrm2
__global__ void k_cycle_init(GmresState *st, double *g, const double *nrm2, int m) {
    if (threadIdx.x != 0) return;
    const double beta = sqrt(*nrm2);
    if (!isfinite(beta)) st->pad[0] = 1;
    st->beta = beta;
    st->est = beta;
    st->j = 0;
    st->active = 0;
    const bool conv = beta <= st->tol;
    st->converged = conv ? 1 : 0;
    st->done = conv ? 1 : 0;
    for (int i = 0; i <= m; ++i) g[i] = 0.0;
    g[0] = beta;
    st->inv = conv ? 0.0 : 1.0 / beta;
}

__global__ void k_cycle_scale(double *__restrict__ V0, double *__restrict__ xa, long long len,
                              const GmresState *__restrict__ st) {
    if (st->done) return;
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= len) return;
    const double v = st->inv * V0[k];
    V0[k] = v;
    xa[k] = v;
}

// y = R^{-1} g over the k = j columns of the finished cycle
__global__ void k_trisolve(const GmresState *__restrict__ st, const double *__restrict__ H,
                           const double *__restrict__ g, double *__restrict__ y, int m) {
    if (threadIdx.x != 0) return;
    const int k = st->j;
    for (int i = k - 1; i >= 0; --i) {
        double acc = g[i];
        for (int l = i + 1; l < k; ++l) acc -= H[(long long)l * (m + 1) + i] * y[l];
        y[i] = acc / H[(long long)i * (m + 1) + i];
    }
}

// x += V[0..k-1] y
__global__ void k_update_x(const double *__restrict__ V, long long len,
                           const GmresState *__restrict__ st, const double *__restrict__ y,
                           double *__restrict__ x) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= len) return;
    const int kc = st->j;
    double s = 0.0;
    for (int jv = 0; jv < kc; ++jv) s += V[(long long)jv * len + k] * y[jv];
    x[k] += 1.0 * s;
}

__global__ void k_copy(const double *__restrict__ a, long long len, double *__restrict__ b) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < len) b[k] = a[k];
}

__global__ void k_residual(const double *__restrict__ b, const double *__restrict__ mx,
                           long long len, double *__restrict__ r) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < len) r[k] = 1.0 * b[k] + -1.0 * mx[k];
}

__global__ void k_zero(double *__restrict__ a, long long len) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < len) a[k] = 0.0;
}

// the kernels of one Arnoldi step (after the matvec of xa into ya)
void enqueue_step(afmpb_ctx *c, bool fp64) {
    GmresEngine &E = c->gm;
    hipStream_t s = c->stream;
    const long long len = E.len;
    const int m = E.m, nblk = (int)E.nblk;
    double *V = c->krylov.p, *w = c->ya.p;
    c->matvec_m(c->xa.p, w, fp64);
    const unsigned gx = grid_for(len, 256);
    const dim3 gp((unsigned)nblk, (unsigned)((m + 1 + VG - 1) / VG));
    k_proj_partial<<<gp, GB, 0, s>>>(V, len, w, nblk, E.st.p, E.part.p);
    KCHK();
    k_proj_final<<<m + 1, GB, 0, s>>>(E.part.p, nblk, E.st.p, E.h1.p);
    KCHK();
    k_proj_update<<<gx, 256, 0, s>>>(V, len, E.st.p, E.h1.p, w);
    KCHK();
    k_proj_partial<<<gp, GB, 0, s>>>(V, len, w, nblk, E.st.p, E.part.p);
    KCHK();
    k_proj_final<<<m + 1, GB, 0, s>>>(E.part.p, nblk, E.st.p, E.h2.p);
    KCHK();
    k_proj_update<<<gx, 256, 0, s>>>(V, len, E.st.p, E.h2.p, w);
    KCHK();
    double *npart = E.part.p + (long long)(m + 1) * nblk;
    k_norm_partial<<<nblk, GB, 0, s>>>(w, len, E.st.p, 1, npart);
    KCHK();
    k_norm_final<<<1, GB, 0, s>>>(npart, nblk, E.st.p, 1, E.h2.p + m + 1);
    KCHK();
    k_givens<<<1, 64, 0, s>>>(E.st.p, E.H.p, E.cs.p, E.sn.p, E.g.p, E.h1.p, E.h2.p,
                               E.h2.p + m + 1, m);
    KCHK();
    k_next_vector<<<gx, 256, 0, s>>>(w, len, E.st.p, V, c->xa.p);
    KCHK();
}

void capture_step(afmpb_ctx *c, bool fp64) {
    GmresEngine &E = c->gm;
    const int i = fp64 ? 0 : 1;
    std::unique_lock<std::shared_mutex> lk(g_capture_mu);
    HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
    try {
        enqueue_step(c, fp64);
    } catch (...) {
        hipGraph_t tmp = nullptr;
        (void)hipStreamEndCapture(c->stream, &tmp);
        if (tmp) (void)hipGraphDestroy(tmp);
        throw;
    }
    HIPCHK(hipStreamEndCapture(c->stream, &E.step_graph[i]));
    HIPCHK(hipGraphInstantiate(&E.step_exec[i], E.step_graph[i], nullptr, nullptr, 0));
}

// ||a||^2 into the device scalar out (no state guard)
void norm2(afmpb_ctx *c, const double *a, double *out) {
    GmresEngine &E = c->gm;
    double *npart = E.part.p + (long long)(E.m + 1) * E.nblk;
    k_norm_partial<<<(unsigned)E.nblk, GB, 0, c->stream>>>(a, E.len, E.st.p, 0, npart);
    KCHK();
    k_norm_final<<<1, GB, 0, c->stream>>>(npart, (int)E.nblk, E.st.p, 0, out);
    KCHK();
}

void to_host(afmpb_ctx *c, int slot) {
    HIPCHK(hipMemcpyAsync(c->gm.host + slot, c->gm.st.p, sizeof(GmresState),
                          hipMemcpyDeviceToHost, c->stream));
}

}  // namespace

GmresEngine::~GmresEngine() { reset(); }

void GmresEngine::reset() {
    std::shared_lock<std::shared_mutex> lk(g_capture_mu);
    for (int i = 0; i < 2; ++i) {
        if (step_exec[i]) (void)hipGraphExecDestroy(step_exec[i]);
        if (step_graph[i]) (void)hipGraphDestroy(step_graph[i]);
        step_exec[i] = nullptr;
        step_graph[i] = nullptr;
        if (ev[i]) (void)hipEventDestroy(ev[i]);
        ev[i] = nullptr;
    }
    if (host) (void)hipHostFree(host);
    host = nullptr;
    m = 0;
    len = 0;
}

void gmres_prepare(afmpb_ctx *c, int m, bool need_fp32) {
    GmresEngine &E = c->gm;
    const long long len = 2 * c->n;
    if (E.m != m || E.len != len) {
        E.reset();
        E.m = m;
        E.len = len;
        E.nblk = (len + GCHUNK - 1) / GCHUNK;
        E.st.alloc(1);
        E.H.alloc((size_t)(m + 1) * m);
        E.cs.alloc(m);
        E.sn.alloc(m);
        E.g.alloc(m + 1);
        E.y.alloc(m);
        E.h1.alloc(m + 2);
        E.h2.alloc(m + 2);
        E.part.alloc((size_t)(m + 2) * E.nblk);
        {
            std::shared_lock<std::shared_mutex> lk(g_capture_mu);
            HIPCHK(hipHostMalloc(reinterpret_cast<void **>(&E.host), 3 * sizeof(GmresState),
                                 hipHostMallocDefault));
            HIPCHK(hipEventCreateWithFlags(&E.ev[0], hipEventDisableTiming));
            HIPCHK(hipEventCreateWithFlags(&E.ev[1], hipEventDisableTiming));
        }
        std::memset(E.host, 0, 3 * sizeof(GmresState));
        if (c->krylov_m < m || c->krylov.n < (size_t)(m + 1) * len) {
            c->krylov.alloc((size_t)(m + 1) * len);
            c->krylov_m = m;
        }
        // a defined state before any capture replays it
        k_zero<<<grid_for(sizeof(GmresState) / sizeof(double), 64), 64, 0, c->stream>>>(
            reinterpret_cast<double *>(E.st.p), sizeof(GmresState) / sizeof(double));
        KCHK();
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    // captured once per precision; profiling runs the same kernels eagerly
    if (!c->prof.on) {
        if (!E.step_exec[0]) capture_step(c, true);
        if (need_fp32 && !E.step_exec[1] && c->prm.precision != AFMPB_FP64) capture_step(c, false);
    }
}

void gmres_set_tol(afmpb_ctx *c, const double *b, double rel_tol, double abs_tol, int slot) {
    GmresEngine &E = c->gm;
    norm2(c, b, E.h1.p + E.m + 1);
    k_set_tol<<<1, 64, 0, c->stream>>>(E.st.p, E.h1.p + E.m + 1, rel_tol, abs_tol);
    KCHK();
    to_host(c, slot);
}

void gmres_cycle_start(afmpb_ctx *c, const double *b, const double *x, bool x_first_zero,
                       bool fp64, int slot) {
    GmresEngine &E = c->gm;
    hipStream_t s = c->stream;
    double *V0 = c->krylov.p;
    const unsigned gx = grid_for(E.len, 256);
    if (x_first_zero) {
        k_copy<<<gx, 256, 0, s>>>(b, E.len, V0);
        KCHK();
    } else {
        k_copy<<<gx, 256, 0, s>>>(x, E.len, c->xa.p);
        KCHK();
        c->matvec_m(c->xa.p, c->ya.p, fp64);
        k_residual<<<gx, 256, 0, s>>>(b, c->ya.p, E.len, V0);
        KCHK();
    }
    norm2(c, V0, E.h1.p + E.m + 1);
    k_cycle_init<<<1, 64, 0, s>>>(E.st.p, E.g.p, E.h1.p + E.m + 1, E.m);
    KCHK();
    k_cycle_scale<<<gx, 256, 0, s>>>(V0, c->xa.p, E.len, E.st.p);
    KCHK();
    to_host(c, slot);
}

void gmres_step(afmpb_ctx *c, bool fp64, int slot) {
    GmresEngine &E = c->gm;
    hipGraphExec_t ex = E.step_exec[fp64 ? 0 : 1];
    if (ex && !c->prof.on) HIPCHK(hipGraphLaunch(ex, c->stream));
    else enqueue_step(c, fp64);
    to_host(c, slot);
}

void gmres_cycle_end(afmpb_ctx *c, double *x) {
    GmresEngine &E = c->gm;
    k_trisolve<<<1, 64, 0, c->stream>>>(E.st.p, E.H.p, E.g.p, E.y.p, E.m);
    KCHK();
    k_update_x<<<grid_for(E.len, 256), 256, 0, c->stream>>>(c->krylov.p, E.len, E.st.p, E.y.p, x);
    KCHK();
}

const GmresState &gmres_status(afmpb_ctx *c, int slot) { return c->gm.host[slot]; }

GmresResult gmres_device(afmpb_ctx *c, const double *b, double *x, bool x_zero, double rel_tol,
                         double abs_tol, int m, int max_restarts, bool fp64,
                         bool final_residual) {
    GmresEngine &E = c->gm;
    gmres_prepare(c, m, !fp64);
    hipStream_t s = c->stream;
    GmresResult R;
    gmres_set_tol(c, b, rel_tol, abs_tol, 2);
    HIPCHK(hipStreamSynchronize(s));
    const double nb = E.host[2].beta;
    R.inner += 1;
    require(std::isfinite(nb), ST_NUMERIC, "non-finite right-hand side");
    if (x_zero) {
        k_zero<<<grid_for(E.len, 256), 256, 0, s>>>(x, E.len);
        KCHK();
    }
    bool first = true;
    for (int cycle = 0; cycle <= max_restarts; ++cycle) {
        gmres_cycle_start(c, b, x, first && x_zero, fp64, 2);
        first = false;
        HIPCHK(hipStreamSynchronize(s));
        const GmresState s0 = E.host[2];
        R.inner += 1;
        R.est = s0.beta;
        require(s0.pad[0] == 0, ST_NUMERIC, "non-finite residual");
        if (s0.converged) { R.converged = true; break; }
        if (cycle > 0) R.restarts += 1;
        // steps with one step of look-ahead: step k+1 is issued before the
        // status of step k is read, unless step k is predicted to end the
        // cycle (its residual estimate extrapolated geometrically from the
        // last two reaches the tolerance): a step issued after the last one
        // still runs its matvec
        int k = 0, issued = 1;
        gmres_step(c, fp64, 0);
        HIPCHK(hipEventRecord(E.ev[0], s));
        GmresState sk{};
        double e1 = s0.beta, e2 = 0.0;        // estimates after steps k-1 and k-2
        for (;;) {
            const bool more = k + 1 < m;
            const bool last = e2 > 0.0 && e1 * (e1 / e2) <= s0.tol;
            if (more && issued == k + 1 && !last) {
                gmres_step(c, fp64, (k + 1) & 1);
                HIPCHK(hipEventRecord(E.ev[(k + 1) & 1], s));
                issued = k + 2;
            }
            HIPCHK(hipEventSynchronize(E.ev[k & 1]));
            sk = E.host[k & 1];
            require(sk.pad[0] == 0, ST_NUMERIC, "non-finite value in the Arnoldi process");
            if (sk.done || !more) {
                if (issued > k + 1) HIPCHK(hipEventSynchronize(E.ev[(k + 1) & 1]));
                break;
            }
            e2 = e1;
            e1 = sk.est;
            ++k;
            if (issued == k) {                // the prediction held the step back
                gmres_step(c, fp64, k & 1);
                HIPCHK(hipEventRecord(E.ev[k & 1], s));
                issued = k + 1;
            }
        }
        const int steps = sk.j;
        R.iterations += steps;
        for (int jj = 0; jj < steps; ++jj) R.inner += 2 * (jj + 1) + 1;
        R.est = sk.est;
        gmres_cycle_end(c, x);
        if (sk.converged) { R.converged = true; break; }
    }
    if (!final_residual) return R;
    // true residual with the FP64 operator
    k_copy<<<grid_for(E.len, 256), 256, 0, s>>>(x, E.len, c->xa.p);
    KCHK();
    c->matvec_m(c->xa.p, c->ya.p, true);
    k_residual<<<grid_for(E.len, 256), 256, 0, s>>>(b, c->ya.p, E.len, c->tmp.p);
    KCHK();
    norm2(c, c->tmp.p, E.h1.p + E.m + 1);
    double rn2 = 0;
    HIPCHK(hipMemcpyAsync(&rn2, E.h1.p + E.m + 1, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double rn = std::sqrt(rn2);
    R.true_rel = nb > 0 ? rn / nb : rn;
    return R;
}

}  // namespace afmpb

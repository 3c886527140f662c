// C ABI of libafmpb: context, molecule setup, matvec, GMRES solve, energy,
// debug views and profiling.  See include/afmpb.h for the contract.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>
#include <cstdlib>
#include <numeric>

#include <cstring>
#include <future>
#include <system_error>

#include "ctx.h"

namespace afmpb {

// ------------------------------- profiling ---------------------------------

int Prof::id_of(const char *name) {
    auto it = index.find(name);
    if (it != index.end()) return it->second;
    int id = (int)entries.size();
    entries.push_back(Entry{name, 0.0, 0});
    index[name] = id;
    return id;
}

hipEvent_t Prof::take() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    return e;
}

void Prof::flush() {
    for (auto &p : pending) {
        int id;
        hipEvent_t a, b;
        std::tie(id, a, b) = p;
        HIPCHK(hipEventSynchronize(b));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, a, b));
        entries[id].ms += ms;
        entries[id].count += 1;
        pool.push_back(a);
        pool.push_back(b);
    }
    pending.clear();
}

Prof::~Prof() {
    for (auto &p : pending) {
        (void)hipEventDestroy(std::get<1>(p));
        (void)hipEventDestroy(std::get<2>(p));
    }
    for (auto e : pool) (void)hipEventDestroy(e);
}

ProfScope::ProfScope(Prof *p, const char *name, hipStream_t st)
    : prof(p), id(-1), s(st), slot(0) {
    if (!prof || !prof->on || (!prof->only.empty() && prof->only != name)) {
        prof = nullptr;
        return;
    }
    id = prof->id_of(name);
    hipEvent_t a = prof->take(), b = prof->take();
    HIPCHK(hipEventRecord(a, s));
    slot = prof->pending.size();
    prof->pending.emplace_back(id, a, b);
    ++prof->open;
}

ProfScope::~ProfScope() {
    if (!prof) return;
    (void)hipEventRecord(std::get<2>(prof->pending[slot]), s);
    if (--prof->open == 0 && prof->pending.size() > 4096) {
        try { prof->flush(); } catch (...) {}
    }
}

// ------------------------------- helpers -----------------------------------

constexpr double E_CHARGE = 1.602176634e-19;
constexpr double AVOGADRO = 6.02214076e23;
constexpr double EPS0 = 8.8541878128e-12;

double unit_scale() {
    // 4 pi * (e^2 N_A / (4 pi eps0)) in kcal A / mol
    double ce = E_CHARGE * E_CHARGE * AVOGADRO / (4.0 * M_PI * EPS0) * 1e10 / 4184.0;
    return 4.0 * M_PI * ce;
}

// What the device setup relies on for memory safety: sizes, finite
// coordinates, triangle indices in range, every node used.
void validate_mesh_indices(long long n, const double *V, long long m, const int *T) {
    require(n >= 4 && m >= 4, ST_MESH, "mesh needs at least 4 nodes and 4 triangles");
    require(n < (1ll << 30) && m < (1ll << 30), ST_INVALID, "mesh too large");
    for (long long i = 0; i < 3 * n; ++i)
        require(std::isfinite(V[i]), ST_INVALID, "non-finite node coordinate");
    std::vector<char> used(n, 0);
    for (long long i = 0; i < 3 * m; ++i) {
        require(T[i] >= 0 && T[i] < n, ST_MESH, "triangle index out of range");
        used[T[i]] = 1;
    }
    for (long long i = 0; i < n; ++i) require(used[i], ST_MESH, "node not used by any triangle");
}

// The rest of the surface conditions (closed, manifold, consistently and
// outward oriented, no duplicate vertex, no zero-area triangle); the indices
// must have passed validate_mesh_indices.
void validate_mesh_topology(long long n, const double *V, long long m, const int *T) {
    std::vector<int> deg(n + 1, 0);
    for (long long i = 0; i < 3 * m; ++i) ++deg[T[i]];
    // duplicate vertices: open-addressing hash of the exact coordinates
    // (-0.0 taken as +0.0, so that equal values hash alike)
    {
        size_t cap = 16;
        while (cap < 2 * (size_t)n) cap <<= 1;
        std::vector<int> slot(cap, -1);
        auto bits = [](double v) {
            if (v == 0.0) v = 0.0;
            unsigned long long u;
            std::memcpy(&u, &v, sizeof u);
            return u;
        };
        for (long long i = 0; i < n; ++i) {
            const double *p = V + 3 * i;
            unsigned long long h = bits(p[0]) * 0x9E3779B97F4A7C15ull;
            h = (h ^ (h >> 29) ^ bits(p[1])) * 0xBF58476D1CE4E5B9ull;
            h = (h ^ (h >> 31) ^ bits(p[2])) * 0x94D049BB133111EBull;
            size_t q = (size_t)(h ^ (h >> 32)) & (cap - 1);
            while (slot[q] >= 0) {
                const double *o = V + 3ll * slot[q];
                require(!(o[0] == p[0] && o[1] == p[1] && o[2] == p[2]), ST_MESH,
                        "duplicate vertex");
                q = (q + 1) & (cap - 1);
            }
            slot[q] = (int)i;
        }
    }
    // directed edges a -> b of every triangle as rows per start node; each
    // directed edge must appear once, and its reverse once (closed, manifold,
    // consistently oriented)
    std::vector<long long> ptr(n + 1, 0);
    for (long long v = 0; v < n; ++v) ptr[v + 1] = ptr[v] + deg[v];
    std::vector<int> nxt(3 * m);
    std::vector<long long> fill(ptr.begin(), ptr.end() - 1);
    for (long long k = 0; k < m; ++k)
        for (int j = 0; j < 3; ++j) {
            const int a = T[3 * k + j], b = T[3 * k + (j + 1) % 3];
            require(a != b, ST_MESH, "degenerate triangle (repeated node)");
            nxt[fill[a]++] = b;
        }
    for (long long v = 0; v < n; ++v) {
        int *r = nxt.data() + ptr[v];
        const long long d = ptr[v + 1] - ptr[v];
        if (d <= 32) {                       // rows are short: insertion sort
            for (long long a = 1; a < d; ++a) {
                const int key = r[a];
                long long b = a - 1;
                while (b >= 0 && r[b] > key) { r[b + 1] = r[b]; --b; }
                r[b + 1] = key;
            }
        } else {
            std::sort(r, r + d);
        }
        for (long long e = 1; e < d; ++e)
            require(r[e] != r[e - 1], ST_MESH, "edge used twice in one direction (non-manifold)");
    }
    for (long long v = 0; v < n; ++v)
        for (long long e = ptr[v]; e < ptr[v + 1]; ++e) {
            const int b = nxt[e];
            require(std::binary_search(nxt.begin() + ptr[b], nxt.begin() + ptr[b + 1], (int)v),
                    ST_MESH, "open surface or inconsistent orientation");
        }
    double asum = 0.0, vol = 0.0;
    std::vector<double> ar(m);
    for (long long k = 0; k < m; ++k) {
        const double *a = V + 3ll * T[3 * k], *b = V + 3ll * T[3 * k + 1], *c = V + 3ll * T[3 * k + 2];
        double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                        e1[0] * e2[1] - e1[1] * e2[0]};
        ar[k] = 0.5 * std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        asum += ar[k];
        vol += (a[0] * (b[1] * c[2] - b[2] * c[1]) + a[1] * (b[2] * c[0] - b[0] * c[2]) +
                a[2] * (b[0] * c[1] - b[1] * c[0])) / 6.0;
    }
    double amean = asum / m;
    for (long long k = 0; k < m; ++k)
        require(ar[k] >= 1e-12 * amean, ST_MESH, "degenerate triangle (zero area)");
    require(vol > 0.0, ST_MESH, "surface encloses non-positive volume (inward orientation?)");
}

}  // namespace afmpb

using namespace afmpb;


namespace afmpb {

int fail(afmpb_ctx *ctx, const Error &e) {
    if (ctx) ctx->err = e.what();
    return e.code;
}

template <class F>
afmpb_status guarded(afmpb_ctx *ctx, F &&f) {
    try {
        // device buffers allocated during the call come from the context's
        // supplier (if it has one)
        AllocScope as(ctx && ctx->has_al ? &ctx->al : nullptr, ctx ? ctx->stream : nullptr);
        f();
        if (ctx) ctx->err.clear();
        return AFMPB_OK;
    } catch (const Error &e) {
        return (afmpb_status)fail(ctx, e);
    } catch (const std::bad_alloc &) {
        if (ctx) ctx->err = "host allocation failed";
        return AFMPB_E_OOM;
    } catch (const std::exception &e) {
        if (ctx) ctx->err = e.what();
        return AFMPB_E_DEVICE;
    }
}

void fill_defaults(afmpb_params &p) {
    p.eps_p = 2.0;
    p.eps_s = 80.0;
    p.kappa = 0.1;
    p.order_p = 8;
    p.leaf_cap = 64;
    p.precision = AFMPB_FP64;
    p.rel_tol = 1e-6;
    p.abs_tol = 0.0;
    p.restart = 80;
    p.max_restarts = 5;
    p.near_eta = 4.0;
    p.m2l_layout = 0;
    p.rhs_fmm = 0;
    p.overlap = 0;
    p.wx_expand = 0;
}

afmpb_params normalise(const afmpb_params &in) {
    afmpb_params p = in;
    auto fin = [](double v) { return std::isfinite(v); };
    require(fin(p.eps_p) && p.eps_p > 0 && fin(p.eps_s) && p.eps_s > 0, ST_INVALID,
            "dielectric constants must be finite and positive");
    require(fin(p.kappa) && p.kappa >= 0, ST_INVALID, "kappa must be finite and >= 0");
    if (p.order_p == 0) p.order_p = 8;
    require(p.order_p >= 2 && p.order_p <= MAXP, ST_INVALID, "order_p must be in [2, 20]");
    if (p.leaf_cap == 0) p.leaf_cap = 64;
    require(p.leaf_cap >= 1, ST_INVALID, "leaf_cap must be >= 1");
    require(p.precision == AFMPB_FP64 || p.precision == AFMPB_FP32_REFINED ||
                p.precision == AFMPB_FP32_BF16M2L_REFINED, ST_INVALID,
            "unknown precision");
    require(fin(p.rel_tol) && p.rel_tol >= 0 && fin(p.abs_tol) && p.abs_tol >= 0, ST_INVALID,
            "tolerances must be finite and >= 0");
    if (p.restart == 0) p.restart = 80;
    require(p.restart >= 1 && p.restart <= 1000, ST_INVALID, "restart must be in [1, 1000]");
    require(p.max_restarts >= 0, ST_INVALID, "max_restarts must be >= 0");
    require(p.m2l_layout >= 0 && p.m2l_layout <= 3, ST_INVALID, "m2l_layout must be 0, 1, 2 or 3");
    require(p.rhs_fmm >= 0 && p.rhs_fmm <= 2, ST_INVALID, "rhs_fmm must be 0, 1 or 2");
    require(p.overlap >= 0 && p.overlap <= 3, ST_INVALID, "overlap must be 0, 1, 2 or 3");
    require(p.wx_expand >= 0, ST_INVALID, "wx_expand must be >= 0");
    require(p.wx_expand < 2 || p.order_p == 6 || p.order_p == 8 || p.order_p == 10 ||
                p.order_p == 14, ST_INVALID, "wx_expand >= 2 needs order_p 6, 8, 10 or 14");
    if (p.near_eta == 0) p.near_eta = 4.0;
    require(fin(p.near_eta) && p.near_eta > 0, ST_INVALID, "near_eta must be > 0");
    return p;
}

// Harmonic-mean point count from which a W entry is taken by expansions
// (0: never).  Automatic is never: on the capsid-scale shell (FP32, p = 8,
// leaf 128) thresholds 24, 48 and 96 moved 49%, 7.8% and 3.9% of the P2P
// pairs and the matvec took 81.5, 58.6 and 58.3 ms against 58.0 ms direct.
int wx_threshold(const afmpb_params &p) {
    return p.wx_expand >= 2 ? p.wx_expand : 0;
}

void ensure_loaded(afmpb_ctx *c) {
    require(c != nullptr, ST_INVALID, "null context");
    require(c->loaded, ST_STATE, "no molecule loaded");
}

__global__ void k_to_f32(const double *a, float *b, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

__global__ void k_finite(const double *a, long long n, int *bad) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(a[i])) atomicOr(bad, 1);
}

template <typename R>
void setup_plan(afmpb_ctx *c, MatvecPlan<R> &mp, DBuf<R> &w, DBuf<R> &far, const R *ndR) {
    const long long n = c->n, K = c->fmm.K, nb = c->tree.nbox;
    const long long ng = c->lists.n_vg * c->lists.m2l_split;   // result slots
    w.alloc((size_t)4 * n);
    if (c->p2p64.n < (size_t)2 * n) c->p2p64.alloc((size_t)2 * n);
    if (c->p2p_part.n < (size_t)c->lists.n_chunks * 128)
        c->p2p_part.alloc((size_t)std::max(c->lists.n_chunks, 1ll) * 128);
    mp.part = c->p2p_part.p;
    if (c->p2p_rpart.n < (size_t)2 * std::max(c->lists.n_rev, 1ll))
        c->p2p_rpart.alloc((size_t)2 * std::max(c->lists.n_rev, 1ll));
    mp.rpart = c->p2p_rpart.p;
    long long widest = 1;
    for (int l = 0; l < c->tree.nlev; ++l)
        widest = std::max(widest, c->tree.level_start[l + 1] - c->tree.level_start[l]);
    const long long KZ = c->fmm.KZ;
    far.alloc((size_t)(2 * nb * K) * 2 + (size_t)std::max(ng, 1ll) * 2 * KZ + 4 * n +
              (size_t)8 * widest * 2 * K);
    mp.n = n;
    mp.tree = &c->tree;
    mp.lists = &c->lists;
    mp.fmm = &c->fmm;
    mp.near = &c->near;
    mp.side = c->side;
    mp.fork = c->ev_fork;
    mp.join = c->ev_join;
    mp.late_p2p = c->prm.overlap == 2;
    mp.serial = c->prm.overlap == 3 || (c->prm.overlap == 0 && n >= SERIAL_MIN_NODES);
    mp.far.p2m_done = mp.late_p2p && !mp.serial ? c->ev_p2m : nullptr;
    if constexpr (sizeof(R) == sizeof(double)) mp.delta = c->near.delta.p;
    else mp.delta = c->near.delta32.p;
    mp.nd64 = c->nodes();
    mp.nd = NodeR<R>{ndR, ndR + n, ndR + 2 * n, ndR + 3 * n, ndR + 4 * n, ndR + 5 * n};
    mp.area = c->nodes().area;
    mp.kappa = c->prm.kappa;
    mp.inv_ebar = c->inv_ebar;
    mp.alpha = c->alpha;
    mp.sf = w.p;
    mp.xp = w.p + 2 * n;
    mp.sh = w.p + n;
    mp.pf = c->p2p64.p;
    mp.ph = c->p2p64.p + n;
    R *f = far.p;
    mp.far.M = f;
    mp.far.Lc = f + 2 * nb * K;
    mp.far.Z = f + 4 * nb * K;         // 16-byte aligned: 4 nb K elements precede it
    mp.far.phi = f + 4 * nb * K + std::max(ng, 1ll) * 2 * KZ;
    mp.far.Mt = mp.far.phi + 4 * n;
    mp.far.bf16_m2l = (sizeof(R) == sizeof(float) &&
                       c->prm.precision == AFMPB_FP32_BF16M2L_REFINED) ? 1 : 0;
}

void check_setup(afmpb_ctx *c);

void load_molecule(afmpb_ctx *c, long long n, const double *xyz, long long m, const int *tri,
                   long long na, const double *axyz, const double *q, const afmpb_params &prm) {
    auto t0 = std::chrono::steady_clock::now();
    auto tp = t0;
    // phase end: wait for the context stream, record the wall time since the
    // last mark as phase ph
    auto mark = [&](int ph) {
        c->sync();
        auto now = std::chrono::steady_clock::now();
        c->ms_phase[ph] = std::chrono::duration<double, std::milli>(now - tp).count();
        tp = now;
    };
    std::fill(c->ms_phase, c->ms_phase + AFMPB_SETUP_PHASES, 0.0);
    c->loaded = false;
    c->gm.reset();            // captured steps refer to the previous molecule's buffers
    validate_mesh_indices(n, xyz, m, tri);
    // the remaining mesh checks run on the host beside the device setup
    // (which needs only valid indices); a failure is raised before the
    // context is marked loaded
    std::future<void> topo;
    try {
        topo = std::async(std::launch::async, validate_mesh_topology, n, xyz, m, tri);
    } catch (const std::system_error &) {
        validate_mesh_topology(n, xyz, m, tri);   // no thread available: in line
    }
    try {
        for (long long i = 0; i < 3 * na; ++i)
            require(std::isfinite(axyz[i]), ST_INVALID, "non-finite atom coordinate");
        for (long long i = 0; i < na; ++i) require(std::isfinite(q[i]), ST_INVALID, "non-finite charge");
        hipStream_t s = c->stream;
        c->prm = prm;
        c->n = n; c->m = m; c->na = na;
        c->ebar = prm.eps_s / prm.eps_p;
        c->inv_ebar = 1.0 / c->ebar;
        c->alpha = 0.5 / c->ebar + 0.5;
        c->V.alloc(3 * n); c->V.upload(xyz, 3 * n, s);
        c->T.alloc(3 * m); c->T.upload(tri, 3 * m, s);
        c->ax.alloc(3 * std::max(na, 1ll)); c->ax.upload(axyz, 3 * na, s);
        c->aq.alloc(std::max(na, 1ll)); c->aq.upload(q, na, s);
        // a0 geometry (caller order)
        c->tri_area.alloc(m); c->tri_n.alloc(3 * m);
        c->inc_ptr.alloc(n + 1); c->inc_tri.alloc(3 * m);
        c->area_c.alloc(n); c->nrm_c.alloc(3 * n); c->rho2_c.alloc(n);
        compute_geometry(c->V.p, c->T.p, n, m, c->tri_area.p, c->tri_n.p, c->inc_ptr.p, c->inc_tri.p,
                         c->area_c.p, c->nrm_c.p, c->rho2_c.p, s);
        mark(0);   // validation, upload, geometry
        // a1 Morton keys and sort
        c->keys.alloc(n); c->perm.alloc(n);
        morton_sort(c->V.p, n, c->keys.p, c->perm.p, c->lo, &c->scale, s);
        c->node64.alloc(8 * n);
        gather_nodes(c->V.p, c->nrm_c.p, c->area_c.p, c->rho2_c.p, c->perm.p, n, c->nodes(), s);
        c->node32.alloc(6 * n);
        k_to_f32<<<grid_for(6 * n, 256), 256, 0, s>>>(c->node64.p, c->node32.p, 6 * n);
        KCHK();
        mark(1);   // keys, sort, node gather
        // a4 near set; its patch-integral corrections (the largest part of
        // the setup) run on the second stream beside everything after it,
        // with device frees held back until they have finished
        c->near = NearSet();
        build_near(c->nodes(), n, prm.near_eta, c->near, s);
        near_coeffs(c->nodes(), n, c->V.p, c->T.p, c->tri_n.p, c->inc_ptr.p, c->inc_tri.p,
                    c->perm.p, prm.kappa, c->ebar, c->near, c->side);
        mark(4);   // near set
        DeferFree held;
        // a2 tree, a3 lists
        c->tree = Tree();
        build_tree(c->keys.p, n, prm.leaf_cap, c->lo, c->scale, c->tree, s);
        c->lists = Lists();
        mark(2);   // tree
        build_lists(c->tree, c->lists, prm.m2l_layout, s, true, true, wx_threshold(prm));
        mark(3);   // lists and P2P / M2L work items
        // translation operators
        c->fmm = Fmm();
        c->p2p64 = DBuf<double>();
        c->p2p_part = DBuf<double>();
        c->p2p_rpart = DBuf<double>();
        build_fmm_operators(c->tree, c->lists, prm.order_p, prm.kappa,
                            prm.precision == AFMPB_FP32_BF16M2L_REFINED, c->fmm, s);
        mark(5);   // translation operators
        setup_plan<double>(c, c->mp64, c->w64, c->far64, c->node64.p);
        setup_plan<float>(c, c->mp32, c->w32, c->far32, c->node32.p);
        c->xa.alloc(2 * n); c->ya.alloc(2 * n); c->bvec.alloc(2 * n);
        c->xsol.alloc(2 * n); c->tmp.alloc(2 * n);
        c->hbuf.alloc(2 * 1024 + 8);
        c->phi_at.alloc(std::max(na, 1ll));
        c->krylov = DBuf<double>();
        c->krylov_m = 0;
        c->sync();
        check_setup(c);
        if (topo.valid()) topo.get();   // rethrows a mesh error
        mark(6);   // work buffers, structural checks, mesh checks
        c->dual = DualTree();
        if (use_dual(c)) build_dual(c);
        mark(7);   // nodes + atoms tree of the right-hand side and energy
        HIPCHK(hipStreamSynchronize(c->side));
        mark(8);   // the rest of the patch-integral corrections
    } catch (...) {
        // a mesh error found meanwhile explains a failure of the device setup
        if (topo.valid()) topo.get();
        throw;
    }
    c->ms_setup = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    c->loaded = true;
}

// Structural checks of every array the matvec kernels index with; a failure
// raises an error here instead of an out-of-range access later.
template <typename T>
std::vector<T> host_copy(const DBuf<T> &b, size_t n, hipStream_t s) {
    std::vector<T> h(n);
    if (n) b.download(h.data(), n, s);
    return h;
}

void check_setup(afmpb_ctx *c) {
    const char *env = std::getenv("AFMPB_CHECK");
    if (env && env[0] == '0') return;
    hipStream_t s = c->stream;
    const long long n = c->n, nb = c->tree.nbox;
    const Tree &t = c->tree;
    const Lists &L = c->lists;
    auto keys = host_copy(c->keys, n, s);
    auto perm = host_copy(c->perm, n, s);
    auto lev = host_copy(t.level, nb, s), par = host_copy(t.parent, nb, s);
    auto cb = host_copy(t.child_begin, nb, s), nc = host_copy(t.n_child, nb, s);
    auto ptb = host_copy(t.pt_begin, nb, s), pte = host_copy(t.pt_end, nb, s);
    c->sync();
    auto bad = [](const char *what) { throw Error(ST_DEVICE, std::string("setup check: ") + what); };
    std::vector<char> seen(n, 0);
    for (long long i = 0; i < n; ++i) {
        if (perm[i] < 0 || perm[i] >= n || seen[perm[i]]) bad("perm is not a permutation");
        seen[perm[i]] = 1;
        if (i && keys[i] < keys[i - 1]) bad("keys not sorted");
    }
    if (nb < 1 || ptb[0] != 0 || pte[0] != n || par[0] != -1 || lev[0] != 0) bad("root box");
    for (long long b = 0; b < nb; ++b) {
        if (ptb[b] < 0 || pte[b] > n || ptb[b] >= pte[b]) bad("box point range");
        if (lev[b] < 0 || lev[b] > 21) bad("box level");
        if (b > 0 && (par[b] < 0 || par[b] >= b || lev[par[b]] != lev[b] - 1)) bad("box parent");
        if (b > 0 && (ptb[b] < ptb[par[b]] || pte[b] > pte[par[b]])) bad("box not inside parent");
        if (nc[b] < 0 || nc[b] > 8) bad("child count");
        if (nc[b] > 0) {
            if (cb[b] <= b || cb[b] + nc[b] > nb) bad("child range");
            if (ptb[cb[b]] != ptb[b] || pte[cb[b] + nc[b] - 1] != pte[b]) bad("children cover");
            for (int k = 0; k < nc[b]; ++k)
                if (par[cb[b] + k] != b) bad("child parent");
        }
    }
    if ((long long)t.level_start.size() != t.nlev + 1 || t.level_start.back() != nb) bad("levels");
    auto csr = [&](const DBuf<int> &ptr, const DBuf<int> &idx, long long cnt, long long lim,
                   const char *what) {
        auto p = host_copy(ptr, nb + 1, s);
        auto ix = host_copy(idx, cnt, s);
        c->sync();
        if (p[0] != 0 || p[nb] != cnt) bad(what);
        for (long long b = 0; b < nb; ++b)
            if (p[b + 1] < p[b]) bad(what);
        for (long long q = 0; q < cnt; ++q)
            if (ix[q] < 0 || ix[q] >= lim) bad(what);
    };
    csr(L.u_ptr, L.u_idx, L.n_u, nb, "U list");
    csr(L.v_ptr, L.v_idx, L.n_v, nb, "V list");
    csr(L.w_ptr, L.w_idx, L.n_w, nb, "W list");
    csr(L.x_ptr, L.x_idx, L.n_x, nb, "X list");
    auto vcls = host_copy(L.v_cls, L.n_v, s);
    auto leaf = host_copy(L.leaf_ids, L.n_leaves, s);
    auto sp = host_copy(L.p2p_ptr, L.n_leaves + 1, s);
    auto src = host_copy(L.p2p_src, L.n_p2p_src, s);
    auto ib = host_copy(L.item_box, L.n_items, s), ibeg = host_copy(L.item_begin, L.n_items, s);
    c->sync();
    for (auto v : vcls) if (v < 0 || v >= 316) bad("V class");
    for (auto b : leaf) if (b < 0 || b >= nb || nc[b] != 0) bad("leaf ids");
    if (sp[0] != 0 || sp[L.n_leaves] != L.n_p2p_src) bad("P2P ptr");
    for (long long i = 0; i < L.n_leaves; ++i) if (sp[i + 1] < sp[i]) bad("P2P ptr");
    for (auto b : src) if (b < 0 || b >= nb) bad("P2P source box");
    for (long long k = 0; k < L.n_items; ++k) {
        if (ib[k] < 0 || ib[k] >= L.n_leaves) bad("P2P item leaf");
        int B = leaf[ib[k]];
        if (ibeg[k] < ptb[B] || ibeg[k] >= pte[B]) bad("P2P item begin");
    }
    {
        auto clo = host_copy(L.ch_lo, L.n_chunks, s), chi = host_copy(L.ch_hi, L.n_chunks, s);
        auto cg = host_copy(L.ch_grp, L.n_chunks, s);
        auto rb = host_copy(L.rng_b, L.n_rng, s), re = host_copy(L.rng_e, L.n_rng, s);
        auto gp = host_copy(L.grp_ptr, L.n_groups + 1, s);
        auto gb = host_copy(L.grp_tbeg, L.n_groups, s), ge = host_copy(L.grp_tend, L.n_groups, s);
        c->sync();
        for (long long k = 0; k < L.n_rng; ++k)
            if (rb[k] < 0 || re[k] > n || rb[k] >= re[k]) bad("P2P source range");
        for (long long k = 0; k < L.n_chunks; ++k) {
            if (clo[k] < 0 || chi[k] > L.n_rng || clo[k] >= chi[k]) bad("P2P chunk span");
            if (cg[k] < 0 || cg[k] >= L.n_groups || k < gp[cg[k]] || k >= gp[cg[k] + 1]) bad("P2P chunk group");
        }
        if (gp[0] != 0 || gp[L.n_groups] != L.n_chunks) bad("P2P group ptr");
        for (long long g = 0; g < L.n_groups; ++g) {
            if (gp[g + 1] <= gp[g]) bad("P2P group without chunks");
            if (gb[g] < 0 || ge[g] > n || gb[g] >= ge[g] || ge[g] - gb[g] > 64) bad("P2P group targets");
        }
        // reverse chunks: each chunk's source stream owns the slots
        // [rev[c], rev[c] + its points); every point's slot list is a set of
        // distinct slots, together all of them
        auto crv = host_copy(L.ch_rev, L.n_chunks, s);
        auto rp = host_copy(L.rev_ptr, n + 1, s);
        auto ri = host_copy(L.rev_idx, std::max(L.n_rev, 1ll), s);
        c->sync();
        for (long long k = 0; k < L.n_chunks; ++k) {
            if (crv[k] < -1) bad("P2P reverse chunk");
            if (crv[k] < 0) continue;
            long long np = 0;
            for (int q = clo[k]; q < chi[k]; ++q) np += re[q] - rb[q];
            if (crv[k] + np > L.n_rev) bad("P2P reverse slots");
        }
        if (rp[0] != 0 || rp[n] != L.n_rev) bad("P2P reverse ptr");
        std::vector<char> used(std::max(L.n_rev, 1ll), 0);
        for (long long p = 0; p < n; ++p) {
            if (rp[p + 1] < rp[p]) bad("P2P reverse ptr");
            for (long long q = rp[p]; q < rp[p + 1]; ++q) {
                if (ri[q] < 0 || ri[q] >= L.n_rev || used[ri[q]]) bad("P2P reverse slot list");
                used[ri[q]] = 1;
            }
        }
    }
    {
        // P2M / L2P items: every leaf once, <= 4 leaves and <= 64 points per
        // item unless the item is a single leaf
        const long long nl = L.n_leaves;
        auto pl = host_copy(L.pm_leaf, nl, s);
        auto pf = host_copy(L.pm_first, L.n_pm, s);
        auto pc = host_copy(L.pm_count, L.n_pm, s);
        auto lb = host_copy(c->tree.pt_begin, c->tree.nbox, s);
        auto le = host_copy(c->tree.pt_end, c->tree.nbox, s);
        auto nch = host_copy(c->tree.n_child, c->tree.nbox, s);
        c->sync();
        std::vector<char> seen(c->tree.nbox, 0);
        for (long long i = 0; i < nl; ++i) {
            if (pl[i] < 0 || pl[i] >= c->tree.nbox || nch[pl[i]] != 0 || seen[pl[i]]) bad("P2M leaf list");
            seen[pl[i]] = 1;
        }
        long long covered = 0;
        for (long long w = 0; w < L.n_pm; ++w) {
            if (pc[w] < 1 || pc[w] > 4 || pf[w] != covered || pf[w] + pc[w] > nl) bad("P2M item");
            long long pts = 0;
            for (int g = 0; g < pc[w]; ++g) pts += le[pl[pf[w] + g]] - lb[pl[pf[w] + g]];
            if (pc[w] > 1 && pts > 64) bad("P2M item points");
            covered += pc[w];
        }
        if (covered != nl) bad("P2M items do not cover the leaves");
    }
    if (L.n_m2l_items > 0) {
        auto iops = host_copy(L.m2l_item_ops, 8 * L.n_m2l_items, s);
        auto ibg = host_copy(L.m2l_item_begin, L.n_m2l_items, s);
        auto icn = host_copy(L.m2l_item_count, L.n_m2l_items, s);
        auto cols = host_copy(L.m2l_cols, L.n_vg, s);
        auto vp = host_copy(L.v_ptr, nb + 1, s);
        auto vcls = host_copy(L.v_cls, L.n_v, s), vtgt = host_copy(L.v_tgt, L.n_v, s);
        std::vector<int> vgp, vgs;
        if (L.m2l_grouped) {
            vgp = host_copy(L.vg_ptr, nb + 1, s);
            vgs = host_copy(L.vg_src, 8 * L.n_vg, s);
        }
        c->sync();
        if (!L.m2l_grouped && L.n_vg != L.n_v) bad("M2L entries");
        long long covered = 0;
        for (long long w = 0; w < L.n_m2l_items; ++w) {
            for (int o = 0; o < 8; ++o)
                if (iops[8 * w + o] < -1 || iops[8 * w + o] >= c->fmm.nkey) bad("M2L item operator");
            if (icn[w] < 1 || icn[w] > 64 || ibg[w] < 0 || ibg[w] + icn[w] > L.n_vg) bad("M2L item range");
            covered += icn[w];
            for (long long q = ibg[w]; q < ibg[w] + icn[w]; ++q) {
                const int g = cols[q];
                if (g < 0 || g >= L.n_vg) bad("M2L item column");
                if (L.m2l_grouped) {
                    for (int o = 0; o < 8; ++o)
                        if (vgs[8 * (long long)g + o] >= 0 && iops[8 * w + o] < 0) bad("M2L child without operator");
                } else {
                    if (iops[8 * w] != (lev[vtgt[g]] - 2) * 316 + vcls[g]) bad("M2L entry operator");
                    for (int o = 1; o < 8; ++o)
                        if (iops[8 * w + o] != -1) bad("M2L entry octant");
                }
            }
        }
        if (covered != L.n_vg) bad("M2L items do not cover the groups");
        std::vector<char> sv(L.n_vg, 0);
        for (long long q = 0; q < L.n_vg; ++q) {
            if (sv[cols[q]]) bad("M2L group permutation");
            sv[cols[q]] = 1;
        }
        if (L.m2l_grouped) {
            if (vgp[0] != 0 || vgp[nb] != L.n_vg) bad("M2L group ptr");
            for (long long B = 0; B < nb; ++B) {
                long long ent = 0;
                for (long long g = vgp[B]; g < vgp[B + 1]; ++g)
                    for (int o = 0; o < 8; ++o) {
                        const int sb = vgs[8 * g + o];
                        if (sb < -1 || sb >= nb) bad("M2L group child");
                        ent += sb >= 0;
                    }
                if (ent != vp[B + 1] - vp[B]) bad("M2L groups do not cover V");
            }
        }
    }
    auto nptr = host_copy(c->near.ptr, n + 1, s);
    auto ncol = host_copy(c->near.col, c->near.nnz, s);
    c->sync();
    if (nptr[0] != 0 || nptr[n] != c->near.nnz) bad("near ptr");
    for (long long p = 0; p < n; ++p) {
        if (nptr[p + 1] <= nptr[p]) bad("near row empty");
        bool self = false;
        for (long long e = nptr[p]; e < nptr[p + 1]; ++e) {
            if (ncol[e] < 0 || ncol[e] >= n) bad("near column");
            if (e > nptr[p] && ncol[e] <= ncol[e - 1]) bad("near row not ascending");
            self |= ncol[e] == p;
        }
        if (!self) bad("near row lacks the diagonal");
    }
}

double host_dot(afmpb_ctx *c, const double *a, const double *b, long long len) {
    if (c->dotv.n < 1) c->dotv.alloc(1);
    dots(a, 0, 1, b, len, c->dotv.p, c->dscratch, c->stream);
    double v;
    HIPCHK(hipMemcpyAsync(&v, c->dotv.p, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    c->sync();
    return v;
}

void rhs_morton(afmpb_ctx *c, double *b) {
    if (c->dual.built) dual_rhs(c, b);
    else rhs(c->nodes(), c->n, c->ax.p, c->aq.p, c->na, c->prm.eps_s, b, c->stream);
}

void energy_sum(afmpb_ctx *c, const double *x_morton, double *out) {
    if (c->dual.built) {
        dual_energy_sum(c, x_morton, out);
        return;
    }
    reaction_potential(c->nodes(), c->n, x_morton, c->ax.p, c->na, c->ebar, c->phi_at.p,
                       c->stream);
    // sum_k q_k phi_k reduced on the device in a fixed block order
    dots(c->aq.p, 0, 1, c->phi_at.p, c->na, out, c->dscratch, c->stream);
}

double energy_of(afmpb_ctx *ctx, const double *x_morton) {
    if (ctx->na == 0) return 0.0;
    if (ctx->dotv.n < 1) ctx->dotv.alloc(1);
    energy_sum(ctx, x_morton, ctx->dotv.p);
    double sum;
    HIPCHK(hipMemcpyAsync(&sum, ctx->dotv.p, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    return 0.5 * sum * unit_scale();
}

}  // namespace afmpb

extern "C" {

afmpb_status afmpb_default_params(afmpb_params *out) {
    if (!out) return AFMPB_E_INVALID;
    fill_defaults(*out);
    return AFMPB_OK;
}

afmpb_status afmpb_create(int device, void *hip_stream, const afmpb_allocator *alloc,
                          afmpb_ctx **out) {
    if (!out) return AFMPB_E_INVALID;
    *out = nullptr;
    if (alloc && (!alloc->alloc || !alloc->free)) return AFMPB_E_INVALID;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return AFMPB_E_INVALID;
    if (hipSetDevice(device) != hipSuccess) return AFMPB_E_DEVICE;
    afmpb_ctx *c = new (std::nothrow) afmpb_ctx();
    if (!c) return AFMPB_E_OOM;
    c->device = device;
    if (alloc) {
        c->al = *alloc;
        c->has_al = true;
    }
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (!c->stream) {
        // a stream of its own: the legacy null stream cannot be captured
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return AFMPB_E_DEVICE;
        }
        c->own_stream = true;
    }
    auto fail_device = [c] {
        if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
        if (c->ev_join) (void)hipEventDestroy(c->ev_join);
        if (c->ev_p2m) (void)hipEventDestroy(c->ev_p2m);
        if (c->side) (void)hipStreamDestroy(c->side);
        hipStream_t own = c->own_stream ? c->stream : nullptr;
        delete c;
        if (own) (void)hipStreamDestroy(own);
        return AFMPB_E_DEVICE;
    };
    try {
        c->noalloc_part = noalloc_scratch(device);
    } catch (const Error &) {
        return fail_device();
    }

    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_p2m, hipEventDisableTiming) != hipSuccess)
        return fail_device();
    *out = c;
    return AFMPB_OK;
}

afmpb_status afmpb_destroy(afmpb_ctx *ctx) {
    if (!ctx) return AFMPB_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipStreamSynchronize(ctx->side);
    (void)hipEventDestroy(ctx->ev_fork);
    (void)hipEventDestroy(ctx->ev_join);
    (void)hipEventDestroy(ctx->ev_p2m);
    (void)hipStreamDestroy(ctx->side);
    hipStream_t own = ctx->own_stream ? ctx->stream : nullptr;
    delete ctx;
    if (own) (void)hipStreamDestroy(own);
    return AFMPB_OK;
}

const char *afmpb_last_error(const afmpb_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

afmpb_status afmpb_set_molecule(afmpb_ctx *ctx, long long n_nodes, const double *xyz,
                                long long n_tri, const int *tri, long long n_atoms,
                                const double *atom_xyz, const double *charge,
                                const double *radius, const afmpb_params *params) {
    (void)radius;
    if (!ctx) return AFMPB_E_INVALID;
    return guarded(ctx, [&] {
        HIPCHK(hipSetDevice(ctx->device));
        ctx->loaded = false;
        require(xyz && tri && params, ST_INVALID, "null argument");
        require(n_atoms >= 0 && (n_atoms == 0 || (atom_xyz && charge)), ST_INVALID,
                "bad atom arrays");
        afmpb_params p = normalise(*params);
        try {
            load_molecule(ctx, n_nodes, xyz, n_tri, tri, n_atoms, atom_xyz, charge, p);
        } catch (...) {
            ctx->loaded = false;
            throw;
        }
    });
}

afmpb_status afmpb_matvec_dev(afmpb_ctx *ctx, const double *x_dev, double *y_dev) {
    if (!ctx) return AFMPB_E_INVALID;
    return guarded(ctx, [&] {
        ensure_loaded(ctx);
        require(x_dev && y_dev, ST_INVALID, "null argument");
        to_morton(x_dev, ctx->perm.p, ctx->n, ctx->xa.p, ctx->stream);
        ctx->matvec_m(ctx->xa.p, ctx->ya.p, false);
        from_morton(ctx->ya.p, ctx->perm.p, ctx->n, y_dev, ctx->stream);
    });
}

afmpb_status afmpb_matvec(afmpb_ctx *ctx, const double *x, double *y) {
    if (!ctx) return AFMPB_E_INVALID;
    return guarded(ctx, [&] {
        ensure_loaded(ctx);
        require(x && y, ST_INVALID, "null argument");
        const long long len = 2 * ctx->n;
        for (long long i = 0; i < len; ++i)
            require(std::isfinite(x[i]), ST_NUMERIC, "non-finite input vector");
        ctx->tmp.upload(x, len, ctx->stream);
        to_morton(ctx->tmp.p, ctx->perm.p, ctx->n, ctx->xa.p, ctx->stream);
        ctx->matvec_m(ctx->xa.p, ctx->ya.p, false);
        from_morton(ctx->ya.p, ctx->perm.p, ctx->n, ctx->tmp.p, ctx->stream);
        ctx->tmp.download(y, len, ctx->stream);
        ctx->sync();
    });
}

afmpb_status afmpb_rhs(afmpb_ctx *ctx, double *b) {
    if (!ctx) return AFMPB_E_INVALID;
    return guarded(ctx, [&] {
        ensure_loaded(ctx);
        require(b != nullptr, ST_INVALID, "null argument");
        rhs_morton(ctx, ctx->bvec.p);
        from_morton(ctx->bvec.p, ctx->perm.p, ctx->n, ctx->tmp.p, ctx->stream);
        ctx->tmp.download(b, 2 * ctx->n, ctx->stream);
        ctx->sync();
    });
}


afmpb_status afmpb_energy(afmpb_ctx *ctx, const double *x, double *energy) {
    if (!ctx) return AFMPB_E_INVALID;
    return guarded(ctx, [&] {
        ensure_loaded(ctx);
        require(x && energy, ST_INVALID, "null argument");
        ctx->tmp.upload(x, 2 * ctx->n, ctx->stream);
        to_morton(ctx->tmp.p, ctx->perm.p, ctx->n, ctx->xa.p, ctx->stream);
        *energy = energy_of(ctx, ctx->xa.p);
    });
}

afmpb_status afmpb_set_precision(afmpb_ctx *ctx, int precision) {
    if (!ctx) return AFMPB_E_INVALID;
    return guarded(ctx, [&] {
        ensure_loaded(ctx);
        require(precision == AFMPB_FP64 || precision == AFMPB_FP32_REFINED ||
                    (precision == AFMPB_FP32_BF16M2L_REFINED && ctx->fmm.Tbh.n > 0),
                ST_INVALID, "precision not available for this molecule");
        ctx->prm.precision = precision;
        ctx->mp32.far.bf16_m2l = precision == AFMPB_FP32_BF16M2L_REFINED ? 1 : 0;
        ctx->gm.reset();      // the captured FP32 step follows the precision
    });
}

afmpb_status afmpb_energy_dev_noalloc(afmpb_ctx *ctx, const double *x_dev, double *energy_dev) {
    if (!ctx) return AFMPB_E_INVALID;
    return guarded(ctx, [&] {
        ensure_loaded(ctx);
        require(x_dev && energy_dev, ST_INVALID, "null argument");
        energy_noalloc(ctx, x_dev, energy_dev);
    });
}

afmpb_status afmpb_solve(afmpb_ctx *ctx, const double *x0, double *f, double *h,
                         double *energy, afmpb_solve_info *info) {
    if (!ctx) return AFMPB_E_INVALID;
    afmpb_solve_info inf{};
    int conv_code = 0;
    afmpb_status st = guarded(ctx, [&] {
        ensure_loaded(ctx);
        auto t0 = std::chrono::steady_clock::now();
        auto ms = [](auto a, auto b) { return std::chrono::duration<double, std::milli>(b - a).count(); };
        const long long n = ctx->n, len = 2 * n;
        hipStream_t s = ctx->stream;
        rhs_morton(ctx, ctx->bvec.p);
        ctx->sync();
        auto t1 = std::chrono::steady_clock::now();
        bool xz = (x0 == nullptr);
        if (!xz) {
            for (long long i = 0; i < len; ++i)
                require(std::isfinite(x0[i]), ST_NUMERIC, "non-finite warm start");
            ctx->tmp.upload(x0, len, s);
            to_morton(ctx->tmp.p, ctx->perm.p, n, ctx->xsol.p, s);
        }
        const afmpb_params &p = ctx->prm;
        GmresResult g;
        if (p.precision == AFMPB_FP64) {
            g = gmres_device(ctx, ctx->bvec.p, ctx->xsol.p, xz, p.rel_tol, p.abs_tol, p.restart,
                             p.max_restarts, true, true);
        } else {
            // iterative refinement: single-precision operator inside, true
            // residual of the double-precision operator outside
            const double nb = std::sqrt(host_dot(ctx, ctx->bvec.p, ctx->bvec.p, len));
            const double tol = p.rel_tol * nb + p.abs_tol;
            if (xz) HIPCHK(hipMemsetAsync(ctx->xsol.p, 0, len * sizeof(double), s));
            DBuf<double> r(len), d(len);
            int steps = 0;
            double rn = nb;
            if (!xz) {
                ctx->matvec_m(ctx->xsol.p, ctx->tmp.p, true);
                axpby(1.0, ctx->bvec.p, -1.0, ctx->tmp.p, len, r.p, s);
                rn = std::sqrt(host_dot(ctx, r.p, r.p, len));
            } else {
                HIPCHK(hipMemcpyAsync(r.p, ctx->bvec.p, len * sizeof(double), hipMemcpyDeviceToDevice, s));
            }
            for (int it = 0; it < 8 && rn > tol; ++it) {
                double inner_rel = std::max(tol / rn, 1e-6);
                GmresResult gi = gmres_device(ctx, r.p, d.p, true, inner_rel, 0.0, p.restart,
                                              p.max_restarts, false, false);
                g.iterations += gi.iterations;
                g.restarts += gi.restarts;
                g.inner += gi.inner;
                axpby(1.0, ctx->xsol.p, 1.0, d.p, len, ctx->xsol.p, s);
                ctx->matvec_m(ctx->xsol.p, ctx->tmp.p, true);
                axpby(1.0, ctx->bvec.p, -1.0, ctx->tmp.p, len, r.p, s);
                rn = std::sqrt(host_dot(ctx, r.p, r.p, len));
                require(std::isfinite(rn), ST_NUMERIC, "non-finite residual");
                ++steps;
            }
            g.converged = rn <= tol;
            g.est = rn;
            g.true_rel = nb > 0 ? rn / nb : rn;
            inf.refinement_steps = steps;
        }
        auto t2 = std::chrono::steady_clock::now();
        double E = energy_of(ctx, ctx->xsol.p);
        auto t3 = std::chrono::steady_clock::now();
        const double us = unit_scale();
        from_morton(ctx->xsol.p, ctx->perm.p, n, ctx->tmp.p, s);
        std::vector<double> xo(len);
        ctx->tmp.download(xo.data(), len, s);
        ctx->sync();
        if (f) for (long long i = 0; i < n; ++i) f[i] = xo[i] * us;
        if (h) for (long long i = 0; i < n; ++i) h[i] = xo[n + i] * us;
        if (energy) *energy = E;
        double nb = std::sqrt(host_dot(ctx, ctx->bvec.p, ctx->bvec.p, len));
        inf.iterations = g.iterations;
        inf.restarts = g.restarts;
        inf.inner_products = g.inner;
        inf.rel_residual_estimate = nb > 0 ? g.est / nb : g.est;
        inf.true_rel_residual = g.true_rel;
        inf.converged = g.converged ? 1 : 0;
        inf.ms_setup = ctx->ms_setup;
        inf.ms_rhs = ms(t0, t1);
        inf.ms_gmres = ms(t1, t2);
        inf.ms_energy = ms(t2, t3);
        inf.ms_total = ms(t0, std::chrono::steady_clock::now());
        if (!g.converged) conv_code = 1;
    });
    if (info) *info = inf;
    if (st == AFMPB_OK && conv_code) {
        ctx->err = "GMRES did not reach the tolerance";
        return AFMPB_E_NOT_CONVERGED;
    }
    return st;
}

afmpb_status afmpb_setup_times(afmpb_ctx *ctx, double *ms) {
    if (!ctx) return AFMPB_E_INVALID;
    return guarded(ctx, [&] {
        ensure_loaded(ctx);
        require(ms != nullptr, ST_INVALID, "null argument");
        for (int i = 0; i < AFMPB_SETUP_PHASES; ++i) ms[i] = ctx->ms_phase[i];
    });
}

afmpb_status afmpb_tree_info(afmpb_ctx *ctx, afmpb_tree_sizes *out) {
    if (!ctx) return AFMPB_E_INVALID;
    return guarded(ctx, [&] {
        ensure_loaded(ctx);
        require(out != nullptr, ST_INVALID, "null argument");
        out->n_nodes = ctx->n;
        out->n_boxes = ctx->tree.nbox;
        out->n_levels = ctx->tree.nlev;
        out->n_u = ctx->lists.n_u;
        out->n_v = ctx->lists.n_v;
        out->n_w = ctx->lists.n_w;
        out->n_x = ctx->lists.n_x;
        out->n_near = ctx->near.nnz;
        out->n_p2p_pairs = ctx->lists.n_p2p_pairs;
        out->n_m2l_pairs = ctx->lists.n_v;
        out->order_p = ctx->prm.order_p;
        out->leaf_cap = ctx->prm.leaf_cap;
        out->n_m2l_slots = ctx->lists.n_vg * ctx->lists.m2l_split;
        out->m2l_layout = ctx->lists.m2l_pairs ? 3 : ctx->lists.m2l_grouped ? 2 : 1;
        out->rhs_mode = ctx->dual.built ? 2 : 1;
        out->rhs_boxes = ctx->dual.built ? ctx->dual.t.nbox : 0;
        out->n_wx_far = ctx->lists.n_wx_far;
        out->n_wx_pairs = ctx->lists.n_wx_pairs;
    });
}

afmpb_status afmpb_debug_tree(afmpb_ctx *ctx, const afmpb_tree_view *o) {
    if (!ctx) return AFMPB_E_INVALID;
    return guarded(ctx, [&] {
        ensure_loaded(ctx);
        require(o != nullptr, ST_INVALID, "null argument");
        hipStream_t s = ctx->stream;
        const long long n = ctx->n, nb = ctx->tree.nbox;
        const Tree &t = ctx->tree;
        const Lists &L = ctx->lists;
        if (o->keys) ctx->keys.download(o->keys, n, s);
        if (o->perm) ctx->perm.download(o->perm, n, s);
        if (o->level) t.level.download(o->level, nb, s);
        if (o->parent) t.parent.download(o->parent, nb, s);
        if (o->child_begin) t.child_begin.download(o->child_begin, nb, s);
        if (o->n_child) t.n_child.download(o->n_child, nb, s);
        if (o->pt_begin) t.pt_begin.download(o->pt_begin, nb, s);
        if (o->pt_end) t.pt_end.download(o->pt_end, nb, s);
        if (o->prefix) t.prefix.download(o->prefix, nb, s);
        if (o->u_ptr) L.u_ptr.download(o->u_ptr, nb + 1, s);
        if (o->u_idx) L.u_idx.download(o->u_idx, L.n_u, s);
        if (o->v_ptr) L.v_ptr.download(o->v_ptr, nb + 1, s);
        if (o->v_idx) L.v_idx.download(o->v_idx, L.n_v, s);
        if (o->v_class) L.v_cls.download(o->v_class, L.n_v, s);
        if (o->w_ptr) L.w_ptr.download(o->w_ptr, nb + 1, s);
        if (o->w_idx) L.w_idx.download(o->w_idx, L.n_w, s);
        if (o->x_ptr) L.x_ptr.download(o->x_ptr, nb + 1, s);
        if (o->x_idx) L.x_idx.download(o->x_idx, L.n_x, s);
        if (o->near_ptr) ctx->near.ptr.download(o->near_ptr, n + 1, s);
        if (o->near_col) ctx->near.col.download(o->near_col, ctx->near.nnz, s);
        if (o->near_delta) ctx->near.delta.download(o->near_delta, 4 * ctx->near.nnz, s);
        ctx->sync();
    });
}

afmpb_status afmpb_profile_enable(afmpb_ctx *ctx, int enable) {
    if (!ctx) return AFMPB_E_INVALID;
    return guarded(ctx, [&] {
        ctx->prof.flush();
        if (enable) {
            for (auto &e : ctx->prof.entries) { e.ms = 0; e.count = 0; }
        }
        ctx->prof.on = enable != 0;
    });
}

afmpb_status afmpb_profile_only(afmpb_ctx *ctx, const char *scope) {
    if (!ctx) return AFMPB_E_INVALID;
    return guarded(ctx, [&] {
        ctx->prof.flush();
        ctx->prof.only = scope ? scope : "";
    });
}

afmpb_status afmpb_profile_read(afmpb_ctx *ctx, int idx, const char **name, double *total_ms,
                                long long *launches) {
    if (!ctx) return AFMPB_E_INVALID;
    afmpb_status st = guarded(ctx, [&] { ctx->prof.flush(); });
    if (st != AFMPB_OK) return st;
    if (idx < 0 || idx >= (int)ctx->prof.entries.size()) return AFMPB_E_INVALID;
    const auto &e = ctx->prof.entries[idx];
    if (name) *name = e.name.c_str();
    if (total_ms) *total_ms = e.ms;
    if (launches) *launches = e.count;
    return AFMPB_OK;
}

}  // extern "C"

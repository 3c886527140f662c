// Fast multipole right-hand side and reaction potential over the nodes and
// atoms held by one octree (see dual.h).  FP64 throughout: both run once per
// solve.
#include <algorithm>

#include "ctx.h"
#include "kernels.h"

namespace afmpb {

namespace {

__global__ void k_concat_points(const double *__restrict__ V, long long n,
                                const double *__restrict__ ax, long long na,
                                double *__restrict__ out) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n + na) return;
    const double *p = i < n ? V + 3 * i : ax + 3 * (i - n);
    out[3 * i] = p[0];
    out[3 * i + 1] = p[1];
    out[3 * i + 2] = p[2];
}

// 1 where the sorted point is a node (combined index < n)
__global__ void k_flag_nodes(const int *__restrict__ perm, long long n, long long ntot,
                             int *__restrict__ flag) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ntot) flag[i] = perm[i] < n ? 1 : 0;
}

// nodes and atoms each in their sorted order: node d (the d-th node of the
// combined order) -> caller node index, atom a -> caller atom index
__global__ void k_split_order(const int *__restrict__ perm, const int *__restrict__ cnode,
                              long long n, long long ntot, int *__restrict__ node_caller,
                              int *__restrict__ atom_caller) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntot) return;
    const int c = perm[i];
    if (c < n) node_caller[cnode[i]] = c;
    else atom_caller[i - cnode[i]] = (int)(c - n);
}

__global__ void k_box_ranges(const int *__restrict__ ptb, const int *__restrict__ pte,
                             const int *__restrict__ cnode, long long nb, int *__restrict__ nb_,
                             int *__restrict__ ne_, int *__restrict__ ab_, int *__restrict__ ae_) {
    long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int p0 = ptb[b], p1 = pte[b];
    nb_[b] = cnode[p0];
    ne_[b] = cnode[p1];
    ab_[b] = p0 - cnode[p0];
    ae_[b] = p1 - cnode[p1];
}

__global__ void k_invert(const int *__restrict__ perm, long long n, int *__restrict__ inv) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) inv[perm[i]] = (int)i;
}

// dual node d: Morton position, coordinates and unit normal
__global__ void k_dual_nodes(const int *__restrict__ node_caller, const int *__restrict__ inv_main,
                             const double *__restrict__ V, const double *__restrict__ nrm,
                             long long n, int *__restrict__ node_main, double *__restrict__ out) {
    long long d = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= n) return;
    const long long c = node_caller[d];
    node_main[d] = inv_main[c];
    for (int a = 0; a < 3; ++a) {
        out[a * n + d] = V[3 * c + a];
        out[(3 + a) * n + d] = nrm[3 * c + a];
    }
}

__global__ void k_dual_atoms(const int *__restrict__ atom_caller, const double *__restrict__ ax,
                             const double *__restrict__ q, long long na, double *__restrict__ out,
                             double *__restrict__ aq) {
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= na) return;
    const long long c = atom_caller[k];
    for (int a = 0; a < 3; ++a) {
        out[a * na + k] = ax[3 * c + a];
        out[(3 + a) * na + k] = 0.0;
    }
    aq[k] = q[c];
}

__global__ void k_fill(double *a, double v, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ void k_scaled_copy(const double *__restrict__ a, double f, long long n,
                              double *__restrict__ b) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = f * a[i];
}

// energy sources at the dual nodes: sf = a f, sh = a h (x in Morton order)
__global__ void k_energy_sources(const int *__restrict__ node_main, const double *__restrict__ area,
                                 const double *__restrict__ x, long long n,
                                 double *__restrict__ sf, double *__restrict__ sh) {
    long long d = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= n) return;
    const long long m = node_main[d];
    sf[d] = area[m] * x[m];
    sh[d] = area[m] * x[n + m];
}

// Near pairs of the two sets: one wave per group of <= 64 targets of a leaf,
// against every source of the boxes that the leaf takes directly (its U, W
// and X lists and the X lists of its ancestors), 64 sources at a time in
// LDS.  Sources carry a charge c and (DIP) a dipole of magnitude d along
// their normal: potential c/r + d (R.n_s)/r^3 and its derivative along the
// target normal, -c (R.n_t)/r^3 + d [(n_t.n_s)/r^3 - 3 (R.n_t)(R.n_s)/r^5],
// with R = target - source (the 1/(4 pi) applied to the sums).
template <bool DIP>
__global__ void __launch_bounds__(64) k_p2p_sets(
    const int *__restrict__ g_leaf, const int *__restrict__ g_b, const int *__restrict__ g_e,
    const int *__restrict__ p2p_ptr, const int *__restrict__ p2p_src,
    const int *__restrict__ sptb, const int *__restrict__ spte, const double *__restrict__ sp,
    long long ns, const double *__restrict__ charge, const double *__restrict__ sf,
    double dip_scale, const double *__restrict__ tp, long long nt, double *__restrict__ out_v,
    double *__restrict__ out_dn) {
    __shared__ double S[8][64];
    const int lane = threadIdx.x;
    const int g = blockIdx.x;
    const int tb = g_b[g], te = g_e[g], leaf = g_leaf[g];
    const long long i = tb + lane;
    const bool act = i < te;
    const long long ii = act ? i : tb;
    const double x = tp[ii], y = tp[nt + ii], z = tp[2 * nt + ii];
    const double tnx = tp[3 * nt + ii], tny = tp[4 * nt + ii], tnz = tp[5 * nt + ii];
    double v = 0.0, dv = 0.0;
    for (int q = p2p_ptr[leaf]; q < p2p_ptr[leaf + 1]; ++q) {
        const int C = p2p_src[q];
        const int sb = sptb[C], se = spte[C];
        for (int s0 = sb; s0 < se; s0 += 64) {
            const int j = s0 + lane;
            const bool in = j < se;
            __syncthreads();
            S[0][lane] = in ? sp[j] : 0.0;
            S[1][lane] = in ? sp[ns + j] : 0.0;
            S[2][lane] = in ? sp[2 * ns + j] : 0.0;
            S[3][lane] = in ? sp[3 * ns + j] : 0.0;
            S[4][lane] = in ? sp[4 * ns + j] : 0.0;
            S[5][lane] = in ? sp[5 * ns + j] : 0.0;
            S[6][lane] = in ? charge[j] : 0.0;
            S[7][lane] = (DIP && in) ? -dip_scale * sf[j] : 0.0;
            __syncthreads();
            const int cnt = min(64, se - s0);
            for (int k = 0; k < cnt; ++k) {
                const double rx = x - S[0][k], ry = y - S[1][k], rz = z - S[2][k];
                const double r2 = (rx * rx + ry * ry) + rz * rz;
                if (r2 == 0.0) continue;          // a target on a source adds nothing
                const double ir = 1.0 / sqrt(r2);
                const double ir3 = ir * ir * ir;
                const double Rt = (rx * tnx + ry * tny) + rz * tnz;
                v += S[6][k] * ir;
                dv -= S[6][k] * Rt * ir3;
                if (DIP) {
                    const double Rs = (rx * S[3][k] + ry * S[4][k]) + rz * S[5][k];
                    const double nn = (tnx * S[3][k] + tny * S[4][k]) + tnz * S[5][k];
                    v += S[7][k] * Rs * ir3;
                    dv += S[7][k] * (nn * ir3 - 3.0 * Rt * Rs * ir3 * ir * ir);
                }
            }
        }
    }
    if (act) {
        out_v[i] = v * INV_4PI;
        out_dn[i] = dv * INV_4PI;
    }
}

// b_f = far potential + near sum, b_h = far normal derivative + near sum,
// scattered from the dual node order to Morton order
__global__ void k_rhs_combine(const int *__restrict__ node_main, const double *__restrict__ phi,
                              const double *__restrict__ pv, const double *__restrict__ pdv,
                              long long n, double *__restrict__ b) {
    long long d = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= n) return;
    const long long m = node_main[d];
    b[m] = phi[d] + pv[d];
    b[n + m] = phi[n + d] + pdv[d];
}

// phi_reac at atom k = ebar (far Laplace potential + near sum), in place
__global__ void k_energy_potential(const double *__restrict__ phi, double ebar, long long na,
                                   double *__restrict__ pv) {
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < na) pv[k] = ebar * (phi[k] + pv[k]);
}

template <typename T>
std::vector<T> down(const DBuf<T> &b, size_t n, hipStream_t s) {
    std::vector<T> h(n);
    if (n) b.download(h.data(), n, s);
    return h;
}

// P2M / L2P items of one set: its leaves in the order of their first point,
// packed as in the matvec (<= 4 consecutive leaves with <= 64 points
// together; a larger leaf alone); leaves without points of the set omitted.
void side_items(const std::vector<int> &leaf, const std::vector<int> &pb,
                const std::vector<int> &pe, DBuf<int> &pm_leaf, DBuf<int> &pm_first,
                DBuf<int> &pm_count, long long &n_pm, long long &pm_max,
                DBuf<int> &pm_bysize, long long &n_leaves, hipStream_t s) {
    std::vector<int> pml, pmf, pmc;
    for (int b : leaf)
        if (pe[b] > pb[b]) pml.push_back(b);
    std::sort(pml.begin(), pml.end(), [&](int a, int b) { return pb[a] < pb[b]; });
    const long long nl = (long long)pml.size();
    n_leaves = nl;
    pm_max = 0;
    for (long long i = 0; i < nl;) {
        int cnt = 1, pts = pe[pml[i]] - pb[pml[i]];
        if (pts <= 64)
            while (i + cnt < nl && cnt < 4 && pts + (pe[pml[i + cnt]] - pb[pml[i + cnt]]) <= 64) {
                pts += pe[pml[i + cnt]] - pb[pml[i + cnt]];
                ++cnt;
            }
        pmf.push_back((int)i);
        pmc.push_back(cnt);
        pm_max = std::max(pm_max, (long long)pts);
        i += cnt;
    }
    n_pm = (long long)pmf.size();
    std::vector<int> pbs(pml);
    std::stable_sort(pbs.begin(), pbs.end(),
                     [&](int a, int b) { return pe[a] - pb[a] > pe[b] - pb[b]; });
    pm_leaf.alloc(std::max(nl, 1ll));
    pm_first.alloc(std::max(n_pm, 1ll));
    pm_count.alloc(std::max(n_pm, 1ll));
    pm_bysize.alloc(std::max(nl, 1ll));
    pm_leaf.upload(pml.data(), pml.size(), s);
    pm_first.upload(pmf.data(), pmf.size(), s);
    pm_count.upload(pmc.data(), pmc.size(), s);
    pm_bysize.upload(pbs.data(), pbs.size(), s);
    HIPCHK(hipStreamSynchronize(s));
}

// Target groups of one set: per leaf (list position i), its targets in
// groups of <= 64.
void side_groups(const std::vector<int> &leaf, const std::vector<int> &pb,
                 const std::vector<int> &pe, DBuf<int> &g_leaf, DBuf<int> &g_b, DBuf<int> &g_e,
                 long long &ng, hipStream_t s) {
    std::vector<int> gl, gb, ge;
    for (size_t i = 0; i < leaf.size(); ++i)
        for (int b0 = pb[leaf[i]]; b0 < pe[leaf[i]]; b0 += 64) {
            gl.push_back((int)i);
            gb.push_back(b0);
            ge.push_back(std::min(b0 + 64, pe[leaf[i]]));
        }
    ng = (long long)gl.size();
    g_leaf.alloc(std::max(ng, 1ll));
    g_b.alloc(std::max(ng, 1ll));
    g_e.alloc(std::max(ng, 1ll));
    g_leaf.upload(gl.data(), gl.size(), s);
    g_b.upload(gb.data(), gb.size(), s);
    g_e.upload(ge.data(), ge.size(), s);
    HIPCHK(hipStreamSynchronize(s));
}

FarSide<double> side_of(const DualTree &D, bool atoms) {
    FarSide<double> f;
    const long long m = atoms ? D.na : D.n;
    const double *p = atoms ? D.atoms.p : D.nodes.p;
    f.ptb = atoms ? D.aptb.p : D.nptb.p;
    f.pte = atoms ? D.apte.p : D.npte.p;
    f.pm_leaf = atoms ? D.apm_leaf.p : D.npm_leaf.p;
    f.pm_first = atoms ? D.apm_first.p : D.npm_first.p;
    f.pm_count = atoms ? D.apm_count.p : D.npm_count.p;
    f.n_pm = atoms ? D.n_apm : D.n_npm;
    f.pm_max_points = atoms ? D.apm_max : D.npm_max;
    f.pm_bysize = atoms ? D.apm_bysize.p : D.npm_bysize.p;
    f.n_pm_leaves = atoms ? D.n_apm_leaves : D.n_npm_leaves;
    f.x = p; f.y = p + m; f.z = p + 2 * m;
    f.nx = p + 3 * m; f.ny = p + 4 * m; f.nz = p + 5 * m;
    f.n = m;
    return f;
}

}  // namespace

bool use_dual(const afmpb_ctx *c) {
    if (c->na == 0) return false;
    if (c->prm.rhs_fmm == 1) return false;
    if (c->prm.rhs_fmm == 2) return true;
    return (double)c->n * (double)c->na >= 17179869184.0;    // 2^34 pairs
}

void build_dual(afmpb_ctx *c) {
    DualTree &D = c->dual;
    D = DualTree();
    hipStream_t s = c->stream;
    const long long n = c->n, na = c->na, ntot = n + na;
    require(ntot < (1ll << 31), ST_INVALID, "too many nodes and atoms for the right-hand side tree");
    D.n = n;
    D.na = na;
    // one Morton order of nodes and atoms together
    DBuf<unsigned long long> keys(ntot);
    DBuf<int> perm(ntot);
    {
        DBuf<double> pts(3 * ntot);
        k_concat_points<<<grid_for(ntot, 256), 256, 0, s>>>(c->V.p, n, c->ax.p, na, pts.p);
        KCHK();
        // the centre of a symmetric surface (where a lone charge often sits)
        // would be the corner of eight boxes at every level, the worst case
        // of the one-box separation (its expansions barely converge): the
        // root is widened so that the centre lies a third of a side inside
        // the boxes of every level
        morton_sort(pts.p, ntot, keys.p, perm.p, D.lo, &D.scale, s, true);
    }
    build_tree(keys.p, ntot, c->prm.leaf_cap, D.lo, D.scale, D.t, s);
    // (its FP64 M2L at order 14 and above runs the grouped kernel: no pairs)
    build_lists(D.t, D.L, 0, s, false, false);
    const long long nb = D.t.nbox;
    // node / atom positions in the combined order and per-box ranges
    DBuf<int> flag(ntot + 1), cnode(ntot + 1), node_caller(n), inv_main(n);
    k_flag_nodes<<<grid_for(ntot, 256), 256, 0, s>>>(perm.p, n, ntot, flag.p);
    KCHK();
    exclusive_scan_i32(flag.p, cnode.p, ntot, s);
    D.atom_caller.alloc(na);
    k_split_order<<<grid_for(ntot, 256), 256, 0, s>>>(perm.p, cnode.p, n, ntot, node_caller.p,
                                                      D.atom_caller.p);
    KCHK();
    D.nptb.alloc(nb); D.npte.alloc(nb); D.aptb.alloc(nb); D.apte.alloc(nb);
    k_box_ranges<<<grid_for(nb, 256), 256, 0, s>>>(D.t.pt_begin.p, D.t.pt_end.p, cnode.p, nb,
                                                   D.nptb.p, D.npte.p, D.aptb.p, D.apte.p);
    KCHK();
    k_invert<<<grid_for(n, 256), 256, 0, s>>>(c->perm.p, n, inv_main.p);
    KCHK();
    D.node_main.alloc(n);
    D.nodes.alloc(6 * n);
    k_dual_nodes<<<grid_for(n, 256), 256, 0, s>>>(node_caller.p, inv_main.p, c->V.p, c->nrm_c.p, n,
                                                  D.node_main.p, D.nodes.p);
    KCHK();
    D.atoms.alloc(6 * na);
    D.aq.alloc(na);
    k_dual_atoms<<<grid_for(na, 256), 256, 0, s>>>(D.atom_caller.p, c->ax.p, c->aq.p, na,
                                                   D.atoms.p, D.aq.p);
    KCHK();
    // items and target groups of each set (host, from the leaf list)
    {
        const long long nl = D.L.n_leaves;
        auto leaf = down(D.L.leaf_ids, nl, s);
        auto nbh = down(D.nptb, nb, s), neh = down(D.npte, nb, s);
        auto abh = down(D.aptb, nb, s), aeh = down(D.apte, nb, s);
        auto sp = down(D.L.p2p_ptr, nl + 1, s);
        auto src = down(D.L.p2p_src, D.L.n_p2p_src, s);
        HIPCHK(hipStreamSynchronize(s));
        // structural checks of what the kernels index with
        for (long long b = 0; b < nb; ++b)
            require(0 <= nbh[b] && nbh[b] <= neh[b] && neh[b] <= n && 0 <= abh[b] &&
                        abh[b] <= aeh[b] && aeh[b] <= na,
                    ST_DEVICE, "right-hand side tree: box ranges");
        require(neh[0] == n && aeh[0] == na && nbh[0] == 0 && abh[0] == 0, ST_DEVICE,
                "right-hand side tree: root ranges");
        require(sp[0] == 0 && sp[nl] == D.L.n_p2p_src, ST_DEVICE, "right-hand side tree: P2P lists");
        for (long long i = 0; i < nl; ++i) {
            require(sp[i + 1] >= sp[i] && leaf[i] >= 0 && leaf[i] < nb, ST_DEVICE,
                    "right-hand side tree: P2P lists");
        }
        for (int b : src) require(b >= 0 && b < nb, ST_DEVICE, "right-hand side tree: P2P source box");
        side_items(leaf, nbh, neh, D.npm_leaf, D.npm_first, D.npm_count, D.n_npm, D.npm_max,
                   D.npm_bysize, D.n_npm_leaves, s);
        side_items(leaf, abh, aeh, D.apm_leaf, D.apm_first, D.apm_count, D.n_apm, D.apm_max,
                   D.apm_bysize, D.n_apm_leaves, s);
        side_groups(leaf, nbh, neh, D.gn_leaf, D.gn_b, D.gn_e, D.n_gn, s);
        side_groups(leaf, abh, aeh, D.ga_leaf, D.ga_b, D.ga_e, D.n_ga, s);
    }
    // Laplace translation operators (kappa = 0) at an order of at least 14:
    // a single charge on the corner of its box (an atom at the centre of a
    // symmetric surface sits on box corners at every level) converges like
    // (sqrt(3)/2 / (2 - sqrt(3)/2))^(p+1), 3e-6 at p = 14
    build_fmm_operators(D.t, D.L, std::max(c->prm.order_p, 14), 0.0, false, D.F, s);
    const long long K = D.F.K, KZ = D.F.KZ, mx = std::max(n, na);
    const long long ng = std::max(D.L.n_vg * D.L.m2l_split, 1ll);
    long long widest = 1;
    for (int l = 0; l < D.t.nlev; ++l)
        widest = std::max(widest, D.t.level_start[l + 1] - D.t.level_start[l]);
    D.far.alloc((size_t)4 * nb * K + (size_t)ng * 2 * KZ + 4 * mx + (size_t)8 * widest * 2 * K);
    D.w.M = D.far.p;
    D.w.Lc = D.far.p + 2 * nb * K;
    D.w.Z = D.far.p + 4 * nb * K;
    D.w.phi = D.w.Z + ng * 2 * KZ;
    D.w.Mt = D.w.phi + 4 * mx;
    D.zero.alloc(mx);
    k_fill<<<grid_for(mx, 256), 256, 0, s>>>(D.zero.p, 0.0, mx);
    KCHK();
    D.srcf.alloc(mx);
    D.srch.alloc(mx);
    D.pv.alloc(mx);
    D.pdv.alloc(mx);
    D.dscratch.alloc(dots_scratch(std::max(na, 1ll), 1));
    HIPCHK(hipStreamSynchronize(s));
    D.built = true;
}

// b (Morton order, [2n]) = right-hand side of Eq. (5) by the FMM pass.
void dual_rhs(afmpb_ctx *c, double *b) {
    DualTree &D = c->dual;
    hipStream_t s = c->stream;
    const FarSide<double> atoms = side_of(D, true), nodes = side_of(D, false);
    k_scaled_copy<<<grid_for(D.na, 256), 256, 0, s>>>(D.aq.p, 1.0 / c->prm.eps_s, D.na, D.srch.p);
    KCHK();
    far_field_sides<double>(D.F, D.t, D.L, atoms, D.zero.p, D.srch.p, nodes, 1.0, D.w, nullptr, s);
    if (D.n_gn > 0) {
        k_p2p_sets<false><<<blocks_ok(D.n_gn, 64), 64, 0, s>>>(
            D.gn_leaf.p, D.gn_b.p, D.gn_e.p, D.L.p2p_ptr.p, D.L.p2p_src.p, D.aptb.p, D.apte.p,
            D.atoms.p, D.na, D.srch.p, nullptr, 0.0, D.nodes.p, D.n, D.pv.p, D.pdv.p);
        KCHK();
    }
    k_rhs_combine<<<grid_for(D.n, 256), 256, 0, s>>>(D.node_main.p, D.w.phi, D.pv.p, D.pdv.p, D.n,
                                                     b);
    KCHK();
}

// out (device scalar) = sum_k q_k phi_reac(r_k) for x (Morton order, [2n]).
void dual_energy_sum(afmpb_ctx *c, const double *x, double *out) {
    DualTree &D = c->dual;
    hipStream_t s = c->stream;
    const FarSide<double> atoms = side_of(D, true), nodes = side_of(D, false);
    k_energy_sources<<<grid_for(D.n, 256), 256, 0, s>>>(D.node_main.p, c->nodes().area, x, D.n,
                                                        D.srcf.p, D.srch.p);
    KCHK();
    far_field_sides<double>(D.F, D.t, D.L, nodes, D.srcf.p, D.srch.p, atoms, c->inv_ebar, D.w,
                            nullptr, s);
    if (D.n_ga > 0) {
        k_p2p_sets<true><<<blocks_ok(D.n_ga, 64), 64, 0, s>>>(
            D.ga_leaf.p, D.ga_b.p, D.ga_e.p, D.L.p2p_ptr.p, D.L.p2p_src.p, D.nptb.p, D.npte.p,
            D.nodes.p, D.n, D.srch.p, D.srcf.p, c->inv_ebar, D.atoms.p, D.na, D.pv.p, D.pdv.p);
        KCHK();
    }
    k_energy_potential<<<grid_for(D.na, 256), 256, 0, s>>>(D.w.phi, c->ebar, D.na, D.pv.p);
    KCHK();
    dots(D.aq.p, 0, 1, D.pv.p, D.na, out, D.dscratch, s);
}

}  // namespace afmpb

// Adaptive octree over Morton-sorted points and the four interaction lists of
// the adaptive FMM (list-1 U, list-2 V, list-3 W, list-4 X; Section 3.2 of
// the paper handles list-3 like list-1 by direct evaluation, as done here for
// both W and X).  Level-synchronous construction, integer geometry only.
#include <algorithm>

#include "geometry.h"

namespace afmpb {

namespace {

constexpr int MAXLEVEL = 21;
constexpr int MAXCOLL = 26;
// M2L blocks (items x kernels x octant shares) wanted per launch
constexpr long long M2L_FILL_BLOCKS = 4096;
// automatic layout: pairs of boxes from this many V entries on (FP32 M2L on
// the 9.7M-node shell at leaf 128, 52 M entries: 26.7 -> 19.3 ms, and at
// leaf 192: 7.46 -> 5.25 ms; on the 100k-atom complex, 7 M entries at
// p = 10: 1.87 -> 2.28 ms)
constexpr long long M2L_PAIR_MIN_ENTRIES = 1ll << 23;
// Grouped M2L from this many V entries on.  Grouping writes ~6x fewer
// result slots but multiplies ~1.4x more padded columns (absent children)
// and balances less evenly over the XCDs; measured on one MI355X it loses
// at 0.22 M entries (FP32 and FP64) and wins at 7.2 M (matvec -10%).
constexpr long long M2L_GROUP_MIN_ENTRIES = 2ll << 20;
constexpr int DFS_STACK = 128;

// ----------------------------- split ---------------------------------------

__global__ void k_split_flags(const unsigned long long *__restrict__ keys, long long n,
                              const int *__restrict__ box_of, const int *__restrict__ ptb,
                              const int *__restrict__ pte, int level, int cap,
                              int *__restrict__ flag) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b = box_of[i];
    int f = 0;
    if (b >= 0 && level < MAXLEVEL && pte[b] - ptb[b] > cap) {
        int sh = 3 * (MAXLEVEL - level - 1);
        f = (i == ptb[b]) || ((keys[i] >> sh) != (keys[i - 1] >> sh));
    }
    flag[i] = f;
}

__global__ void k_make_children(const unsigned long long *__restrict__ keys, long long n,
                                int *__restrict__ box_of, const int *__restrict__ flag,
                                const int *__restrict__ pos, const int *__restrict__ ptb_old,
                                const int *__restrict__ pte_old, int level, int cap,
                                long long base, long long capb, int *lev,
                                unsigned long long *prefix, int *parent, int *ptb,
                                int *child_begin, int *n_child, int *err) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b = box_of[i];
    bool split = b >= 0 && level < MAXLEVEL && pte_old[b] - ptb_old[b] > cap;
    if (!split) {
        box_of[i] = -1;
        return;
    }
    int sh = 3 * (MAXLEVEL - level - 1);
    long long id = base + pos[i] + flag[i] - 1;
    if (id < base || id >= capb) {
        atomicOr(err, 1);
        box_of[i] = -1;
        return;
    }
    if (flag[i]) {
        lev[id] = level + 1;
        prefix[id] = keys[i] >> sh;
        parent[id] = b;
        ptb[id] = (int)i;
        child_begin[id] = -1;
        n_child[id] = 0;
    }
    box_of[i] = (int)id;
}

__global__ void k_finish_children(long long base, long long cnt, const int *__restrict__ parent,
                                  const int *__restrict__ ptb, int *pte, int *child_begin,
                                  int *n_child) {
    long long k = base + (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= base + cnt) return;
    int p = parent[k];
    bool last = (k + 1 == base + cnt) || parent[k + 1] != p;
    pte[k] = last ? pte[p] : ptb[k + 1];
    if (k == base || parent[k - 1] != p) {
        child_begin[p] = (int)k;
        int c = 1;
        while (k + c < base + cnt && parent[k + c] == p) ++c;
        n_child[p] = c;
    }
}

__global__ void k_box_centers(long long nbox, const int *__restrict__ lev,
                              const unsigned long long *__restrict__ prefix, double lx, double ly,
                              double lz, double inv_scale, double *center) {
    long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    int l = lev[b];
    unsigned long long p = prefix[b];
    long long ia[3] = {0, 0, 0};
    for (int k = 0; k < l; ++k)
        for (int a = 0; a < 3; ++a) ia[a] |= (long long)((p >> (3 * k + a)) & 1ull) << k;
    long long side = 1ll << (MAXLEVEL - l);
    const double lo[3] = {lx, ly, lz};
    for (int a = 0; a < 3; ++a)
        center[3 * b + a] = lo[a] + ((double)(ia[a] * side) + 0.5 * (double)side) * inv_scale;
}

template <typename T>
void grow(DBuf<T> &buf, size_t need, size_t used, hipStream_t s) {
    if (buf.n >= need) return;
    DBuf<T> nb(std::max(need, buf.n * 2));
    if (used) HIPCHK(hipMemcpyAsync(nb.p, buf.p, used * sizeof(T), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    buf = std::move(nb);
}

// ----------------------------- lists ---------------------------------------

struct TreeView {
    const int *lev, *parent, *cb, *nc, *ptb, *pte;
    const unsigned long long *prefix;
    const int *coll, *ncoll;
};

__device__ inline void anchor_of(const TreeView &t, int b, long long a[3]) {
    int l = t.lev[b];
    unsigned long long p = t.prefix[b];
    a[0] = a[1] = a[2] = 0;
    for (int k = 0; k < l; ++k)
        for (int d = 0; d < 3; ++d) a[d] |= (long long)((p >> (3 * k + d)) & 1ull) << k;
    for (int d = 0; d < 3; ++d) a[d] <<= (MAXLEVEL - l);
}

__device__ inline bool is_ancestor(const TreeView &t, int a, int b) {
    int la = t.lev[a], lb = t.lev[b];
    return la < lb && (t.prefix[b] >> (3 * (lb - la))) == t.prefix[a];
}

// Distinct boxes, neither an ancestor of the other, closed cubes touching.
__device__ inline bool adj(const TreeView &t, int a, int b) {
    if (a == b || is_ancestor(t, a, b) || is_ancestor(t, b, a)) return false;
    long long pa[3], pb[3];
    anchor_of(t, a, pa);
    anchor_of(t, b, pb);
    long long sa = 1ll << (MAXLEVEL - t.lev[a]), sb = 1ll << (MAXLEVEL - t.lev[b]);
    for (int d = 0; d < 3; ++d)
        if (!(pa[d] <= pb[d] + sb && pb[d] <= pa[d] + sa)) return false;
    return true;
}

__device__ inline bool is_leaf(const TreeView &t, int b) { return t.nc[b] == 0; }

__global__ void k_colleagues(TreeView t, long long begin, long long end, int *coll, int *ncoll) {
    long long B = begin + (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= end) return;
    int c[MAXCOLL];
    int nc = 0;
    int P = t.parent[B];
    if (P >= 0) {
        // siblings, then children of the parent's colleagues
        for (int k = -1; k < t.ncoll[P]; ++k) {
            int Q = (k < 0) ? P : t.coll[(long long)P * MAXCOLL + k];
            for (int j = 0; j < t.nc[Q]; ++j) {
                int C = t.cb[Q] + j;
                if (C != B && adj(t, (int)B, C) && nc < MAXCOLL) c[nc++] = C;
            }
        }
    }
    for (int i = 1; i < nc; ++i) {
        int v = c[i], j = i - 1;
        while (j >= 0 && c[j] > v) { c[j + 1] = c[j]; --j; }
        c[j + 1] = v;
    }
    for (int i = 0; i < nc; ++i) coll[B * MAXCOLL + i] = c[i];
    ncoll[B] = nc;
}

struct CountEmit {
    int u = 0, v = 0, w = 0;
    __device__ void U(int) { ++u; }
    __device__ void V(int) { ++v; }
    __device__ void W(int) { ++w; }
};

struct FillEmit {
    int *u, *v, *w, *ue, *ve, *we;
    int *err;
    __device__ void U(int c) { if (u < ue) *u++ = c; else atomicOr(err, 1); }
    __device__ void V(int c) { if (v < ve) *v++ = c; else atomicOr(err, 1); }
    __device__ void W(int c) { if (w < we) *w++ = c; else atomicOr(err, 1); }
};

// Enumerates U(B) (leaf), W(B) (leaf) and V(B) (level >= 2) in an arbitrary
// order; rows are sorted afterwards.  Returns false on stack overflow.
template <class E>
__device__ bool enumerate(const TreeView &t, int B, E &e) {
    bool ok = true;
    if (is_leaf(t, B)) {
        e.U(B);
        int stack[DFS_STACK];
        for (int k = 0; k < t.ncoll[B]; ++k) {
            int C = t.coll[(long long)B * MAXCOLL + k];
            if (is_leaf(t, C)) { e.U(C); continue; }
            int sp = 0;
            stack[sp++] = C;
            while (sp > 0) {
                int Q = stack[--sp];
                for (int j = 0; j < t.nc[Q]; ++j) {
                    int D = t.cb[Q] + j;
                    if (adj(t, B, D)) {
                        if (is_leaf(t, D)) e.U(D);
                        else if (sp < DFS_STACK) stack[sp++] = D;
                        else ok = false;
                    } else {
                        e.W(D);
                    }
                }
            }
        }
        // coarser adjacent leaves: leaf colleagues of proper ancestors
        for (int A = t.parent[B]; A >= 0; A = t.parent[A])
            for (int k = 0; k < t.ncoll[A]; ++k) {
                int C = t.coll[(long long)A * MAXCOLL + k];
                if (is_leaf(t, C) && adj(t, B, C)) e.U(C);
            }
    }
    if (t.lev[B] >= 2) {
        int P = t.parent[B];
        for (int k = 0; k < t.ncoll[P]; ++k) {
            int Q = t.coll[(long long)P * MAXCOLL + k];
            for (int j = 0; j < t.nc[Q]; ++j) {
                int C = t.cb[Q] + j;
                if (!adj(t, B, C)) e.V(C);
            }
        }
    }
    return ok;
}

__global__ void k_list_count(TreeView t, long long nbox, int *cu, int *cv, int *cw, int *err) {
    long long B = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= nbox) return;
    CountEmit e;
    if (!enumerate(t, (int)B, e)) atomicOr(err, 1);
    cu[B] = e.u;
    cv[B] = e.v;
    cw[B] = e.w;
}

__global__ void k_list_fill(TreeView t, long long nbox, const int *pu, const int *pv,
                            const int *pw, int *iu, int *iv, int *iw, int *err) {
    long long B = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= nbox) return;
    FillEmit e{iu + pu[B], iv + pv[B], iw + pw[B], iu + pu[B + 1], iv + pv[B + 1],
               iw + pw[B + 1], err};
    enumerate(t, (int)B, e);
    if (e.u != e.ue || e.v != e.ve || e.w != e.we) atomicOr(err, 2);
}

// Offset class of C relative to B: rank of (anchor_C - anchor_B)/side in
// [-3,3]^3 minus [-1,1]^3, ascending lexicographic (dx, dy, dz).
// Rank of the offset (o0, o1, o2) in [-3,3]^3 minus [-1,1]^3, lexicographic.
__host__ __device__ inline int offset_class(int o0, int o1, int o2) {
    const int full = ((o0 + 3) * 7 + (o1 + 3)) * 7 + (o2 + 3);
    // number of excluded (|o|_inf <= 1) positions that precede `full`
    int excl = 0;
    for (int x = -1; x <= 1; ++x)
        for (int y = -1; y <= 1; ++y)
            for (int z = -1; z <= 1; ++z)
                if (((x + 3) * 7 + (y + 3)) * 7 + (z + 3) < full) ++excl;
    return full - excl;
}

__global__ void k_v_class(TreeView t, long long nbox, const int *vptr, const int *vidx,
                          int *vcls, int *vtgt) {
    long long B = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= nbox) return;
    long long ab[3];
    anchor_of(t, (int)B, ab);
    long long side = 1ll << (MAXLEVEL - t.lev[B]);
    for (int q = vptr[B]; q < vptr[B + 1]; ++q) {
        long long ac[3];
        anchor_of(t, vidx[q], ac);
        int d[3];
        for (int a = 0; a < 3; ++a) d[a] = (int)((ac[a] - ab[a]) / side);
        vcls[q] = offset_class(d[0], d[1], d[2]);
        vtgt[q] = (int)B;
    }
}

// M2L groups: the entries of V(B) that are children of one colleague C of
// B's parent P.  They are contiguous in the ascending list (siblings have
// consecutive box indices).  A group's bucket is (level, offset d = C - P in
// [-1,1]^3, octant b of B); the child in octant c sits at offset 2 d + c - b
// from B, so one bucket has one operator per child octant.  Buckets are
// ordered by d before b: the 8 buckets of one d use only 27 offsets, so
// consecutive work items share their operators in cache.
__global__ void k_vg_count(long long nbox, const int *parent, const int *vptr, const int *vidx,
                           int *cnt) {
    long long B = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= nbox) return;
    int n = 0;
    for (int q = vptr[B]; q < vptr[B + 1]; ++q)
        if (q == vptr[B] || parent[vidx[q]] != parent[vidx[q - 1]]) ++n;
    cnt[B] = n;
}

__global__ void k_vg_fill(TreeView t, long long nbox, const int *vptr, const int *vidx,
                          const int *vgptr, int *src, unsigned long long *key, int *idx,
                          int *err) {
    long long B = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= nbox) return;
    long long ab[3];
    anchor_of(t, (int)B, ab);
    const long long side = 1ll << (MAXLEVEL - t.lev[B]);
    const int b = (int)(t.prefix[B] & 7ull);
    int g = vgptr[B] - 1;
    for (int q = vptr[B]; q < vptr[B + 1]; ++q) {
        const int sb = vidx[q];
        const int c = (int)(t.prefix[sb] & 7ull);
        if (q == vptr[B] || t.parent[sb] != t.parent[vidx[q - 1]]) {
            ++g;
            if (g >= vgptr[B + 1]) { atomicOr(err, 8); return; }
            for (int j = 0; j < 8; ++j) src[8 * (long long)g + j] = -1;
            long long ac[3];
            anchor_of(t, sb, ac);
            int dk = 0;
            for (int a = 0; a < 3; ++a) {
                const int o = (int)((ac[a] - ab[a]) / side);
                const int d2 = o + ((b >> a) & 1) - ((c >> a) & 1);
                if (d2 < -2 || d2 > 2 || (d2 & 1)) { atomicOr(err, 8); return; }
                dk = 3 * dk + d2 / 2 + 1;
            }
            key[g] = (unsigned long long)((t.lev[B] - 2) * 216 + dk * 8 + b);
            idx[g] = g;
        }
        if (src[8 * (long long)g + c] != -1) { atomicOr(err, 8); return; }
        src[8 * (long long)g + c] = sb;
    }
    if (g + 1 != vgptr[B + 1]) atomicOr(err, 8);
}

// Pair key of every grouped-layout group (before its keys are sorted):
// (level, colleague offset) and the target's parent, and (group, octant).
__global__ void k_pair_keys(long long nbox, const int *parent, const int *vgptr,
                            const unsigned long long *gkey, unsigned long long *pkey, int *pval) {
    long long B = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= nbox) return;
    for (int g = vgptr[B]; g < vgptr[B + 1]; ++g) {
        pkey[g] = (gkey[g] >> 3) * (unsigned long long)nbox + (unsigned long long)parent[B];
        pval[g] = 8 * g + (int)(gkey[g] & 7ull);
    }
}

__global__ void k_x_count(long long nbox, const int *wptr, const int *widx, int *cnt) {
    long long C = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (C >= nbox) return;
    for (int q = wptr[C]; q < wptr[C + 1]; ++q) atomicAdd(&cnt[widx[q]], 1);
}

__global__ void k_x_fill(long long nbox, const int *wptr, const int *widx, const int *xptr,
                         int *cursor, int *xidx, int *err) {
    long long C = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (C >= nbox) return;
    for (int q = wptr[C]; q < wptr[C + 1]; ++q) {
        int B = widx[q];
        if (B < 0 || B >= nbox) { atomicOr(err, 4); continue; }
        int o = xptr[B] + atomicAdd(&cursor[B], 1);
        if (o >= xptr[B + 1]) { atomicOr(err, 4); continue; }
        xidx[o] = (int)C;
    }
}

__global__ void k_leaf_flags(TreeView t, long long nbox, int *flag) {
    long long B = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= nbox) return;
    flag[B] = is_leaf(t, (int)B);
}

__global__ void k_leaf_collect(long long nbox, const int *flag, const int *pos, int *leaf_ids) {
    long long B = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= nbox) return;
    if (flag[B]) leaf_ids[pos[B]] = (int)B;
}

// Per leaf: number of P2P source boxes, work items, and point pairs.
__global__ void k_p2p_count(TreeView t, long long nleaf, const int *leaf_ids, const int *uptr,
                            const int *uidx, const int *wptr, const int *widx, const int *xptr,
                            const int *xidx, int *nsrc, int *nitem, long long *npairs,
                            long long *srcpts) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nleaf) return;
    int B = leaf_ids[i];
    int cnt = (uptr[B + 1] - uptr[B]) + (wptr[B + 1] - wptr[B]);
    long long src_pts = 0;
    for (int q = uptr[B]; q < uptr[B + 1]; ++q) src_pts += t.pte[uidx[q]] - t.ptb[uidx[q]];
    for (int q = wptr[B]; q < wptr[B + 1]; ++q) src_pts += t.pte[widx[q]] - t.ptb[widx[q]];
    for (int A = B; A >= 0; A = t.parent[A]) {
        cnt += xptr[A + 1] - xptr[A];
        for (int q = xptr[A]; q < xptr[A + 1]; ++q) src_pts += t.pte[xidx[q]] - t.ptb[xidx[q]];
    }
    long long npt = t.pte[B] - t.ptb[B];
    nsrc[i] = cnt;
    nitem[i] = (int)((npt + 63) / 64);
    npairs[i] = npt * src_pts - npt;
    srcpts[i] = src_pts;
}

__global__ void k_p2p_fill(TreeView t, long long nleaf, const int *leaf_ids, const int *uptr,
                           const int *uidx, const int *wptr, const int *widx, const int *xptr,
                           const int *xidx, const int *sptr, int *src, const int *iptr,
                           int *item_box, int *item_begin, int *err) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nleaf) return;
    int B = leaf_ids[i];
    int o = sptr[i];
    const int oe = sptr[i + 1];
    for (int q = uptr[B]; q < uptr[B + 1]; ++q) { if (o < oe) src[o] = uidx[q]; ++o; }
    for (int q = wptr[B]; q < wptr[B + 1]; ++q) { if (o < oe) src[o] = widx[q]; ++o; }
    for (int A = B; A >= 0; A = t.parent[A])
        for (int q = xptr[A]; q < xptr[A + 1]; ++q) { if (o < oe) src[o] = xidx[q]; ++o; }
    if (o != oe) atomicOr(err, 8);
    int k = iptr[i];
    const int ke = iptr[i + 1];
    for (int b = t.ptb[B]; b < t.pte[B]; b += 64) {
        if (k < ke) { item_box[k] = (int)i; item_begin[k] = b; }
        ++k;
    }
    if (k != ke) atomicOr(err, 8);
}

__global__ void k_m2l_keys(long long nv, const int *vtgt, const int *vcls, const int *lev,
                           unsigned long long *keys, int *idx) {
    long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nv) return;
    keys[q] = (unsigned long long)((lev[vtgt[q]] - 2) * 316 + vcls[q]);
    idx[q] = (int)q;
}

template <typename T>
T read_scalar(const T *p, hipStream_t s) {
    T v;
    HIPCHK(hipMemcpyAsync(&v, p, sizeof(T), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return v;
}

}  // namespace

void build_tree(const unsigned long long *keys, long long n, int cap, const double lo[3],
                double scale, Tree &t, hipStream_t s) {
    size_t capb = (size_t)(2 * n / std::max(cap, 1) + 64);
    t.level.alloc(capb); t.parent.alloc(capb); t.child_begin.alloc(capb);
    t.n_child.alloc(capb); t.pt_begin.alloc(capb); t.pt_end.alloc(capb);
    t.prefix.alloc(capb);
    {
        // copies on this context's stream, waited for before the host values
        // (on this stack frame) go out of scope; no legacy-stream operation,
        // so other threads may capture graphs meanwhile
        const int root_i[6] = {0, -1, -1, 0, 0, (int)n};  // level parent cb nc ptb pte
        const unsigned long long z = 0;
        int *dst[6] = {t.level.p, t.parent.p, t.child_begin.p, t.n_child.p, t.pt_begin.p,
                       t.pt_end.p};
        for (int i = 0; i < 6; ++i)
            HIPCHK(hipMemcpyAsync(dst[i], &root_i[i], sizeof(int), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(t.prefix.p, &z, sizeof(z), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    DBuf<int> box_of(n), flag(n + 1), pos(n + 1), gerr(1);
    box_of.zero(n, s);
    gerr.zero(1, s);
    t.level_start.assign(1, 0);
    t.level_start.push_back(1);
    long long nbox = 1;
    for (int l = 0; l < MAXLEVEL; ++l) {
        k_split_flags<<<grid_for(n, 256), 256, 0, s>>>(keys, n, box_of.p, t.pt_begin.p,
                                                       t.pt_end.p, l, cap, flag.p);
        KCHK();
        exclusive_scan_i32(flag.p, pos.p, n, s);
        long long cnt = read_scalar(pos.p + n, s);
        if (cnt == 0) break;
        size_t need = (size_t)(nbox + cnt);
        grow(t.level, need, nbox, s); grow(t.parent, need, nbox, s);
        grow(t.child_begin, need, nbox, s); grow(t.n_child, need, nbox, s);
        grow(t.pt_begin, need, nbox, s); grow(t.pt_end, need, nbox, s);
        grow(t.prefix, need, nbox, s);
        k_make_children<<<grid_for(n, 256), 256, 0, s>>>(
            keys, n, box_of.p, flag.p, pos.p, t.pt_begin.p, t.pt_end.p, l, cap, nbox,
            (long long)std::min({t.level.n, t.prefix.n, t.parent.n, t.pt_begin.n, t.pt_end.n,
                                 t.child_begin.n, t.n_child.n}),
            t.level.p, t.prefix.p, t.parent.p, t.pt_begin.p, t.child_begin.p, t.n_child.p,
            gerr.p);
        KCHK();
        k_finish_children<<<grid_for(cnt, 256), 256, 0, s>>>(nbox, cnt, t.parent.p, t.pt_begin.p,
                                                             t.pt_end.p, t.child_begin.p,
                                                             t.n_child.p);
        KCHK();
        nbox += cnt;
        t.level_start.push_back(nbox);
    }
    require(read_scalar(gerr.p, s) == 0, ST_DEVICE, "tree split: box index out of range");
    t.nbox = nbox;
    t.nlev = (int)t.level_start.size() - 1;
    t.center.alloc(3 * nbox);
    k_box_centers<<<grid_for(nbox, 256), 256, 0, s>>>(nbox, t.level.p, t.prefix.p, lo[0], lo[1],
                                                      lo[2], 1.0 / scale, t.center.p);
    KCHK();
    t.side.resize(t.nlev);
    for (int l = 0; l < t.nlev; ++l) t.side[l] = (double)(1ll << (MAXLEVEL - l)) / scale;
    HIPCHK(hipStreamSynchronize(s));
}

// Operator key of target octant b and source octant c of a pair at
// colleague offset d (level lev), or -1 when the two children are adjacent.
static int pair_op(int lev, const int d[3], int b, int c) {
    int o[3], far = 0;
    for (int a = 0; a < 3; ++a) {
        o[a] = 2 * d[a] + ((c >> a) & 1) - ((b >> a) & 1);
        far |= o[a] < -1 || o[a] > 1;
    }
    return far ? (lev - 2) * 316 + offset_class(o[0], o[1], o[2]) : -1;
}

// Pair layout from the grouped one: groups sorted by (level, colleague
// offset, parent of the target); a run of equal keys is one pair (P, C),
// its groups the target octants.  gkey: the groups' keys by group index.
void build_pairs(const Tree &t, Lists &L, const unsigned long long *gkey, long long ng,
                 hipStream_t s) {
    const long long nb = t.nbox;
    DBuf<unsigned long long> pk(ng), tk(ng);
    DBuf<int> pv(ng), tv(ng);
    k_pair_keys<<<grid_for(nb, 128), 128, 0, s>>>(nb, t.parent.p, L.vg_ptr.p, gkey, pk.p, pv.p);
    KCHK();
    const unsigned long long maxkey = (unsigned long long)(t.nlev * 27 + 1) * (unsigned long long)nb;
    int bits = 1;
    while (bits < 64 && (maxkey >> bits)) ++bits;
    radix_sort_pairs(pk.p, pv.p, tk.p, tv.p, ng, bits, s);
    std::vector<unsigned long long> hk(ng);
    std::vector<int> hv(ng), hs((size_t)8 * ng);
    pk.download(hk.data(), ng, s);
    pv.download(hv.data(), ng, s);
    L.vg_src.download(hs.data(), (size_t)8 * ng, s);
    HIPCHK(hipStreamSynchronize(s));
    std::vector<int> psrc, pslot, iops, ib, ic;
    long long np = 0;
    unsigned long long cur = ~0ull;
    int lev = 0, d[3] = {0, 0, 0};
    for (long long i = 0; i < ng;) {
        const unsigned long long ld = hk[i] / (unsigned long long)nb;
        if (ib.empty() || ld != cur || ic.back() == 64) {       // a new item
            cur = ld;
            lev = (int)(ld / 27) + 2;
            const int dk = (int)(ld % 27);
            d[0] = dk / 9 - 1; d[1] = (dk / 3) % 3 - 1; d[2] = dk % 3 - 1;
            ib.push_back((int)np);
            ic.push_back(0);
            for (int b = 0; b < 8; ++b)
                for (int c = 0; c < 8; ++c) iops.push_back(pair_op(lev, d, b, c));
        }
        int src[8], slot[8];
        for (int o = 0; o < 8; ++o) src[o] = slot[o] = -1;
        long long j = i;
        for (; j < ng && hk[j] == hk[i]; ++j) {
            const int g = hv[j] >> 3, b = hv[j] & 7;
            require(slot[b] < 0, ST_DEVICE, "M2L pairs: two groups of one target octant");
            slot[b] = g;
            for (int c = 0; c < 8; ++c) {
                const int sb = hs[(size_t)8 * g + c];
                if (sb < 0) continue;
                require(pair_op(lev, d, b, c) >= 0, ST_DEVICE, "M2L pairs: adjacent V entry");
                require(src[c] < 0 || src[c] == sb, ST_DEVICE, "M2L pairs: sources disagree");
                src[c] = sb;
            }
        }
        psrc.insert(psrc.end(), src, src + 8);
        pslot.insert(pslot.end(), slot, slot + 8);
        ++np;
        ++ic.back();
        i = j;
    }
    L.n_pairs = np;
    L.n_pr_items = (long long)ib.size();
    L.pr_src.alloc(psrc.size());
    L.pr_slot.alloc(pslot.size());
    L.pr_item_ops.alloc(iops.size());
    L.pr_item_begin.alloc(ib.size());
    L.pr_item_count.alloc(ic.size());
    L.pr_src.upload(psrc.data(), psrc.size(), s);
    L.pr_slot.upload(pslot.data(), pslot.size(), s);
    L.pr_item_ops.upload(iops.data(), iops.size(), s);
    L.pr_item_begin.upload(ib.data(), ib.size(), s);
    L.pr_item_count.upload(ic.data(), ic.size(), s);
    HIPCHK(hipStreamSynchronize(s));   // host vectors must outlive the copies
}

void build_lists(const Tree &t, Lists &L, int m2l_layout, hipStream_t s, bool p2p_chunks,
                 bool auto_pairs, int wx_tau) {
    const long long nb = t.nbox;
    L.coll.alloc((size_t)nb * MAXCOLL);
    L.ncoll.alloc(nb);
    L.ncoll.zero(nb, s);
    TreeView tv{t.level.p, t.parent.p, t.child_begin.p, t.n_child.p, t.pt_begin.p, t.pt_end.p,
                t.prefix.p, L.coll.p, L.ncoll.p};
    for (int l = 1; l < t.nlev; ++l) {
        long long b = t.level_start[l], e = t.level_start[l + 1];
        k_colleagues<<<grid_for(e - b, 128), 128, 0, s>>>(tv, b, e, L.coll.p, L.ncoll.p);
        KCHK();
    }
    DBuf<int> cu(nb + 1), cv(nb + 1), cw(nb + 1), err(1);
    err.zero(1, s);
    k_list_count<<<grid_for(nb, 128), 128, 0, s>>>(tv, nb, cu.p, cv.p, cw.p, err.p);
    KCHK();
    require(read_scalar(err.p, s) == 0, ST_INVALID, "tree too deep for list traversal");
    L.u_ptr.alloc(nb + 1); L.v_ptr.alloc(nb + 1); L.w_ptr.alloc(nb + 1);
    exclusive_scan_i32(cu.p, L.u_ptr.p, nb, s);
    exclusive_scan_i32(cv.p, L.v_ptr.p, nb, s);
    exclusive_scan_i32(cw.p, L.w_ptr.p, nb, s);
    L.n_u = read_scalar(L.u_ptr.p + nb, s);
    L.n_v = read_scalar(L.v_ptr.p + nb, s);
    L.n_w = read_scalar(L.w_ptr.p + nb, s);
    L.u_idx.alloc(L.n_u); L.v_idx.alloc(L.n_v); L.w_idx.alloc(L.n_w);
    L.v_cls.alloc(L.n_v); L.v_tgt.alloc(L.n_v);
    k_list_fill<<<grid_for(nb, 128), 128, 0, s>>>(tv, nb, L.u_ptr.p, L.v_ptr.p, L.w_ptr.p,
                                                  L.u_idx.p, L.v_idx.p, L.w_idx.p, err.p);
    KCHK();
    require(read_scalar(err.p, s) == 0, ST_DEVICE, "list fill out of range");
    sort_rows_i32(L.u_ptr.p, L.u_idx.p, nb, s);
    sort_rows_i32(L.v_ptr.p, L.v_idx.p, nb, s);
    sort_rows_i32(L.w_ptr.p, L.w_idx.p, nb, s);
    k_v_class<<<grid_for(nb, 128), 128, 0, s>>>(tv, nb, L.v_ptr.p, L.v_idx.p, L.v_cls.p,
                                                L.v_tgt.p);
    KCHK();
    // X = transpose of W
    DBuf<int> cx(nb + 1), cur(nb + 1);
    cx.zero(nb + 1, s);
    cur.zero(nb + 1, s);
    k_x_count<<<grid_for(nb, 256), 256, 0, s>>>(nb, L.w_ptr.p, L.w_idx.p, cx.p);
    KCHK();
    L.x_ptr.alloc(nb + 1);
    exclusive_scan_i32(cx.p, L.x_ptr.p, nb, s);
    L.n_x = read_scalar(L.x_ptr.p + nb, s);
    L.x_idx.alloc(L.n_x);
    k_x_fill<<<grid_for(nb, 256), 256, 0, s>>>(nb, L.w_ptr.p, L.w_idx.p, L.x_ptr.p, cur.p,
                                               L.x_idx.p, err.p);
    KCHK();
    require(read_scalar(err.p, s) == 0, ST_DEVICE, "X-list fill out of range");
    sort_rows_i32(L.x_ptr.p, L.x_idx.p, nb, s);
    // leaves and P2P work
    DBuf<int> lflag(nb + 1), lpos(nb + 1);
    k_leaf_flags<<<grid_for(nb, 256), 256, 0, s>>>(tv, nb, lflag.p);
    KCHK();
    exclusive_scan_i32(lflag.p, lpos.p, nb, s);
    L.n_leaves = read_scalar(lpos.p + nb, s);
    L.leaf_ids.alloc(L.n_leaves);
    k_leaf_collect<<<grid_for(nb, 256), 256, 0, s>>>(nb, lflag.p, lpos.p, L.leaf_ids.p);
    KCHK();
    const long long nl = L.n_leaves;
    DBuf<int> nsrc(nl + 1), nitem(nl + 1), iptr(nl + 1);
    DBuf<long long> npairs(nl + 1), srcpts(nl + 1);
    (void)srcpts;
    k_p2p_count<<<grid_for(nl, 128), 128, 0, s>>>(tv, nl, L.leaf_ids.p, L.u_ptr.p, L.u_idx.p,
                                                  L.w_ptr.p, L.w_idx.p, L.x_ptr.p, L.x_idx.p,
                                                  nsrc.p, nitem.p, npairs.p, srcpts.p);
    KCHK();
    L.p2p_ptr.alloc(nl + 1);
    exclusive_scan_i32(nsrc.p, L.p2p_ptr.p, nl, s);
    exclusive_scan_i32(nitem.p, iptr.p, nl, s);
    exclusive_scan_i64(npairs.p, npairs.p, nl, s);
    L.n_p2p_src = read_scalar(L.p2p_ptr.p + nl, s);
    L.n_items = read_scalar(iptr.p + nl, s);
    L.n_p2p_pairs = read_scalar(npairs.p + nl, s);
    L.p2p_src.alloc(L.n_p2p_src);
    L.item_box.alloc(L.n_items);
    L.item_begin.alloc(L.n_items);
    k_p2p_fill<<<grid_for(nl, 128), 128, 0, s>>>(tv, nl, L.leaf_ids.p, L.u_ptr.p, L.u_idx.p,
                                                 L.w_ptr.p, L.w_idx.p, L.x_ptr.p, L.x_idx.p,
                                                 L.p2p_ptr.p, L.p2p_src.p, iptr.p,
                                                 L.item_box.p, L.item_begin.p, err.p);
    KCHK();
    require(read_scalar(err.p, s) == 0, ST_DEVICE, "P2P task fill out of range");
    {
        // Balanced P2P chunks.  The point pairs of the U, W and X lists are
        // symmetric (U(B) holds C iff U(C) holds B; X is the transpose of W),
        // so every unordered pair of point sets is evaluated once: leaf B
        // takes its own points (one-directional, the pair p = t excluded),
        // the leaves of U(B) after B and the boxes of W(B); those are
        // reverse chunks, whose sources also receive the targets'
        // contributions (the X-list side of W, and the other side of U).
        // Source point ranges (touching ranges merged) are cut into spans of
        // at most P2P_CHUNK points per lane copy; every (target group, span)
        // is one work item.
        constexpr int P2P_CHUNK = 256;
        std::vector<int> leaf(nl), ptb_h(nb), pte_h(nb);
        std::vector<int> uptr(nb + 1), uidx(std::max(L.n_u, 1ll)), wptr(nb + 1), widx(std::max(L.n_w, 1ll));
        L.leaf_ids.download(leaf.data(), nl, s);
        t.pt_begin.download(ptb_h.data(), nb, s);
        t.pt_end.download(pte_h.data(), nb, s);
        L.u_ptr.download(uptr.data(), nb + 1, s);
        L.u_idx.download(uidx.data(), L.n_u, s);
        L.w_ptr.download(wptr.data(), nb + 1, s);
        L.w_idx.download(widx.data(), L.n_w, s);
        HIPCHK(hipStreamSynchronize(s));
        const long long npts = pte_h[0];
        if (p2p_chunks) {
        std::vector<int> rb, re, clo, chi, cgrp, gptr, gtb, gte, crev;
        std::vector<std::pair<int, int>> r, far;   // far: W entries (B, C) by expansions
        long long nrev = 0, pairs = 0, far_pairs = 0;
        // cut merged ranges into spans of <= budget points: returns the span
        // boundaries (indices into rb/re)
        auto spans = [&](std::vector<std::pair<int, int>> &m, long long budget) {
            std::vector<long long> cut{(long long)rb.size()};
            long long acc = 0;
            for (auto &x : m) {
                int b = x.first;
                while (b < x.second) {
                    int e = (int)std::min<long long>(x.second, b + (budget - acc));
                    rb.push_back(b);
                    re.push_back(e);
                    acc += e - b;
                    b = e;
                    if (acc == budget) { cut.push_back((long long)rb.size()); acc = 0; }
                }
            }
            if ((long long)rb.size() > cut.back()) cut.push_back((long long)rb.size());
            return cut;
        };
        auto npts_of = [&](long long lo, long long hi) {
            long long c = 0;
            for (long long k = lo; k < hi; ++k) c += re[k] - rb[k];
            return c;
        };
        for (long long i = 0; i < nl; ++i) {
            const int B = leaf[i];
            // replicated lanes take proportionally more sources per chunk
            const long long budget =
                (long long)P2P_CHUNK * p2p_replicas(std::min(64, pte_h[B] - ptb_h[B]));
            std::vector<std::pair<int, int>> self{{ptb_h[B], pte_h[B]}};
            const std::vector<long long> cs = spans(self, budget);
            r.clear();
            for (int q = uptr[B]; q < uptr[B + 1]; ++q)
                if (uidx[q] > B) r.emplace_back(ptb_h[uidx[q]], pte_h[uidx[q]]);
            for (int q = wptr[B]; q < wptr[B + 1]; ++q) {
                const int C = widx[q];
                const long long nbp = pte_h[B] - ptb_h[B], ncp = pte_h[C] - ptb_h[C];
                // harmonic mean 2 nb nc / (nb + nc) >= tau
                if (wx_tau > 0 && ncp > 0 && 2 * nbp * ncp >= (long long)wx_tau * (nbp + ncp)) {
                    far.emplace_back(B, C);
                    far_pairs += 2 * nbp * ncp;
                    continue;
                }
                r.emplace_back(ptb_h[C], pte_h[C]);
            }
            std::sort(r.begin(), r.end());
            std::vector<std::pair<int, int>> m;
            for (auto &x : r) {
                if (!m.empty() && x.first <= m.back().second) m.back().second = std::max(m.back().second, x.second);
                else m.push_back(x);
            }
            const std::vector<long long> cr = spans(m, budget);
            for (int tb = ptb_h[B]; tb < pte_h[B]; tb += 64) {
                const int te = std::min(tb + 64, pte_h[B]);
                gptr.push_back((int)clo.size());
                gtb.push_back(tb);
                gte.push_back(te);
                pairs += (long long)(te - tb) * (pte_h[B] - ptb_h[B] - 1);
                for (size_t k = 0; k + 1 < cs.size(); ++k) {
                    clo.push_back((int)cs[k]);
                    chi.push_back((int)cs[k + 1]);
                    cgrp.push_back((int)gtb.size() - 1);
                    crev.push_back(-1);
                }
                for (size_t k = 0; k + 1 < cr.size(); ++k) {
                    const long long np = npts_of(cr[k], cr[k + 1]);
                    clo.push_back((int)cr[k]);
                    chi.push_back((int)cr[k + 1]);
                    cgrp.push_back((int)gtb.size() - 1);
                    crev.push_back((int)nrev);
                    nrev += np;
                    pairs += 2 * (long long)(te - tb) * np;
                }
            }
        }
        gptr.push_back((int)clo.size());
        require(rb.size() < (1ull << 31) && clo.size() < (1ull << 31) && nrev < (1ll << 31),
                ST_INVALID, "too many P2P chunks");
        require(pairs + far_pairs == L.n_p2p_pairs, ST_DEVICE,
                "P2P tasks do not cover the U/W/X point pairs exactly once");
        L.n_p2p_pairs = pairs;
        L.wx_tau = wx_tau;
        L.n_wx_far = (long long)far.size();
        L.n_wx_pairs = far_pairs;
        if (!far.empty()) {
            // M2P side: far W boxes per leaf (the loop visits leaves in
            // order, so `far` is grouped by B), one item per 64 points
            std::vector<int> fwp(nb + 1, 0), fwi(far.size()), mleaf, mtb;
            for (auto &e : far) ++fwp[e.first + 1];
            for (long long b = 0; b < nb; ++b) fwp[b + 1] += fwp[b];
            for (size_t q = 0; q < far.size(); ++q) fwi[q] = far[q].second;
            for (long long b = 0; b < nb; ++b)
                if (fwp[b + 1] > fwp[b])
                    for (int tb = ptb_h[b]; tb < pte_h[b]; tb += 64) {
                        mleaf.push_back((int)b);
                        mtb.push_back(tb);
                    }
            // P2L side: the transpose, far X leaves per box
            std::vector<std::pair<int, int>> fx(far.size());
            for (size_t q = 0; q < far.size(); ++q) fx[q] = {far[q].second, far[q].first};
            std::sort(fx.begin(), fx.end());
            std::vector<int> fxp(nb + 1, 0), fxi(fx.size()), pbox;
            for (auto &e : fx) ++fxp[e.first + 1];
            for (long long b = 0; b < nb; ++b) fxp[b + 1] += fxp[b];
            for (size_t q = 0; q < fx.size(); ++q) fxi[q] = fx[q].second;
            for (long long b = 0; b < nb; ++b)
                if (fxp[b + 1] > fxp[b]) pbox.push_back((int)b);
            auto put = [&](DBuf<int> &d, const std::vector<int> &h) {
                d.alloc(h.size());
                d.upload(h.data(), h.size(), s);
            };
            put(L.fw_ptr, fwp);
            put(L.fw_idx, fwi);
            put(L.m2p_leaf, mleaf);
            put(L.m2p_tb, mtb);
            put(L.fx_ptr, fxp);
            put(L.fx_idx, fxi);
            put(L.p2l_box, pbox);
            L.n_m2p_items = (long long)mleaf.size();
            L.n_p2l_boxes = (long long)pbox.size();
            HIPCHK(hipStreamSynchronize(s));
        }
        // reverse slots of every point, in chunk order (CSR over points)
        {
            std::vector<int> cnt(npts + 1, 0), rptr(npts + 1), ridx(std::max(nrev, 1ll));
            for (size_t c = 0; c < clo.size(); ++c)
                if (crev[c] >= 0)
                    for (int k = clo[c]; k < chi[c]; ++k)
                        for (int p = rb[k]; p < re[k]; ++p) ++cnt[p];
            rptr[0] = 0;
            for (long long p = 0; p < npts; ++p) rptr[p + 1] = rptr[p] + cnt[p];
            std::vector<int> cur(rptr.begin(), rptr.end() - 1);
            for (size_t c = 0; c < clo.size(); ++c) {
                if (crev[c] < 0) continue;
                int slot = crev[c];
                for (int k = clo[c]; k < chi[c]; ++k)
                    for (int p = rb[k]; p < re[k]; ++p) ridx[cur[p]++] = slot++;
            }
            L.n_rev = nrev;
            L.rev_ptr.alloc(npts + 1);
            L.rev_idx.alloc(ridx.size());
            L.rev_ptr.upload(rptr.data(), rptr.size(), s);
            L.rev_idx.upload(ridx.data(), ridx.size(), s);
            HIPCHK(hipStreamSynchronize(s));   // host vectors must outlive the copies
        }
        L.n_rng = (long long)rb.size();
        L.n_chunks = (long long)clo.size();
        L.n_groups = (long long)gtb.size();
        L.rng_b.alloc(L.n_rng); L.rng_e.alloc(L.n_rng);
        L.ch_lo.alloc(L.n_chunks); L.ch_hi.alloc(L.n_chunks); L.ch_grp.alloc(L.n_chunks);
        L.ch_rev.alloc(L.n_chunks);
        L.ch_rev.upload(crev.data(), crev.size(), s);
        L.grp_ptr.alloc(L.n_groups + 1); L.grp_tbeg.alloc(L.n_groups); L.grp_tend.alloc(L.n_groups);
        L.rng_b.upload(rb.data(), rb.size(), s); L.rng_e.upload(re.data(), re.size(), s);
        L.ch_lo.upload(clo.data(), clo.size(), s); L.ch_hi.upload(chi.data(), chi.size(), s);
        L.ch_grp.upload(cgrp.data(), cgrp.size(), s);
        L.grp_ptr.upload(gptr.data(), gptr.size(), s);
        L.grp_tbeg.upload(gtb.data(), gtb.size(), s); L.grp_tend.upload(gte.data(), gte.size(), s);
        HIPCHK(hipStreamSynchronize(s));   // host vectors must outlive the copies
        }
        // P2M / L2P items: leaves sorted by first point, packed
        std::vector<int> pml(leaf.begin(), leaf.end()), pmf, pmc;
        std::sort(pml.begin(), pml.end(), [&](int a, int b) { return ptb_h[a] < ptb_h[b]; });
        for (long long i = 0; i < nl;) {
            int cnt = 1, pts = pte_h[pml[i]] - ptb_h[pml[i]];
            if (pts <= 64)
                while (i + cnt < nl && cnt < 4 &&
                       pts + (pte_h[pml[i + cnt]] - ptb_h[pml[i + cnt]]) <= 64) {
                    pts += pte_h[pml[i + cnt]] - ptb_h[pml[i + cnt]];
                    ++cnt;
                }
            pmf.push_back((int)i);
            pmc.push_back(cnt);
            L.pm_max_points = std::max(L.pm_max_points, (long long)pts);
            i += cnt;
        }
        L.n_pm = (long long)pmf.size();
        std::vector<int> pbs(pml);
        std::stable_sort(pbs.begin(), pbs.end(), [&](int a, int b) {
            return pte_h[a] - ptb_h[a] > pte_h[b] - ptb_h[b];
        });
        L.n_pm_leaves = nl;
        L.pm_leaf.alloc(nl); L.pm_first.alloc(L.n_pm); L.pm_count.alloc(L.n_pm);
        L.pm_bysize.alloc(std::max(nl, 1ll));
        L.pm_leaf.upload(pml.data(), pml.size(), s);
        L.pm_first.upload(pmf.data(), pmf.size(), s);
        L.pm_count.upload(pmc.data(), pmc.size(), s);
        L.pm_bysize.upload(pbs.data(), pbs.size(), s);
        HIPCHK(hipStreamSynchronize(s));   // host vectors must outlive the copies
    }
    // M2L work items.  Per entry: items of <= 64 V entries of one (level,
    // offset class), each entry its own group with its one operator in
    // octant slot 0 and its own result slot (target-major list order).
    // Grouped (large trees): groups bucketed by (level, colleague offset,
    // octant) into items of <= 64.
    const long long nv = L.n_v;
    L.levels_with_v.clear();
    L.n_m2l_items = 0;
    L.n_vg = 0;
    L.m2l_split = 1;
    L.m2l_grouped = m2l_layout == 0 ? nv >= M2L_GROUP_MIN_ENTRIES : m2l_layout >= 2;
    L.m2l_pairs = m2l_layout == 0 ? auto_pairs && nv >= M2L_PAIR_MIN_ENTRIES : m2l_layout == 3;
    L.n_pairs = L.n_pr_items = 0;
    if (nv == 0) {
        L.vg_ptr.alloc(nb + 1);
        L.vg_ptr.zero(nb + 1, s);
    } else if (!L.m2l_grouped) {
        L.n_vg = nv;
        L.m2l_cols.alloc(nv);
        DBuf<unsigned long long> keys(nv), tk(nv);
        DBuf<int> tvv(nv);
        k_m2l_keys<<<grid_for(nv, 256), 256, 0, s>>>(nv, L.v_tgt.p, L.v_cls.p, t.level.p,
                                                     keys.p, L.m2l_cols.p);
        KCHK();
        radix_sort_pairs(keys.p, L.m2l_cols.p, tk.p, tvv.p, nv, 16, s);
        std::vector<unsigned long long> hk(nv);
        keys.download(hk.data(), nv, s);
        HIPCHK(hipStreamSynchronize(s));
        std::vector<int> iops, ib, ic;
        long long i = 0;
        while (i < nv) {
            long long j = i;
            while (j < nv && hk[j] == hk[i] && j - i < 64) ++j;
            iops.push_back((int)hk[i]);
            for (int c = 1; c < 8; ++c) iops.push_back(-1);
            ib.push_back((int)i);
            ic.push_back((int)(j - i));
            const int lev = (int)(hk[i] / 316) + 2;
            if (L.levels_with_v.empty() || L.levels_with_v.back() != lev)
                L.levels_with_v.push_back(lev);
            i = j;
        }
        L.n_m2l_items = (long long)ib.size();
        L.m2l_item_ops.alloc(iops.size());
        L.m2l_item_begin.alloc(ib.size());
        L.m2l_item_count.alloc(ib.size());
        L.m2l_item_ops.upload(iops.data(), iops.size(), s);
        L.m2l_item_begin.upload(ib.data(), ib.size(), s);
        L.m2l_item_count.upload(ic.data(), ic.size(), s);
        HIPCHK(hipStreamSynchronize(s));   // host vectors must outlive the copies
    } else {
        L.vg_ptr.alloc(nb + 1);
        DBuf<int> cg(nb + 1);
        err.zero(1, s);
        k_vg_count<<<grid_for(nb, 128), 128, 0, s>>>(nb, t.parent.p, L.v_ptr.p, L.v_idx.p, cg.p);
        KCHK();
        exclusive_scan_i32(cg.p, L.vg_ptr.p, nb, s);
        const long long ng = read_scalar(L.vg_ptr.p + nb, s);
        L.n_vg = ng;
        L.vg_src.alloc((size_t)8 * ng);
        L.m2l_cols.alloc(ng);
        DBuf<unsigned long long> keys(ng), tk(ng);
        DBuf<int> tvv(ng);
        k_vg_fill<<<grid_for(nb, 128), 128, 0, s>>>(tv, nb, L.v_ptr.p, L.v_idx.p, L.vg_ptr.p,
                                                    L.vg_src.p, keys.p, L.m2l_cols.p, err.p);
        KCHK();
        require(read_scalar(err.p, s) == 0, ST_DEVICE, "M2L groups inconsistent with V lists");
        if (L.m2l_pairs) build_pairs(t, L, keys.p, ng, s);
        radix_sort_pairs(keys.p, L.m2l_cols.p, tk.p, tvv.p, ng, 16, s);
        std::vector<unsigned long long> hk(ng);
        keys.download(hk.data(), ng, s);
        HIPCHK(hipStreamSynchronize(s));
        std::vector<int> iops, ib, ic;
        long long i = 0;
        while (i < ng) {
            long long j = i;
            while (j < ng && hk[j] == hk[i] && j - i < 64) ++j;
            const int key = (int)hk[i], lev = key / 216 + 2, dk = (key % 216) / 8, b = key % 8;
            const int d[3] = {dk / 9 - 1, (dk / 3) % 3 - 1, dk % 3 - 1};
            for (int c = 0; c < 8; ++c) {
                int o[3], far = 0;
                for (int a = 0; a < 3; ++a) {
                    o[a] = 2 * d[a] + ((c >> a) & 1) - ((b >> a) & 1);
                    far |= o[a] < -1 || o[a] > 1;
                }
                iops.push_back(far ? (lev - 2) * 316 + offset_class(o[0], o[1], o[2]) : -1);
            }
            ib.push_back((int)i);
            ic.push_back((int)(j - i));
            if (L.levels_with_v.empty() || L.levels_with_v.back() != lev)
                L.levels_with_v.push_back(lev);
            i = j;
        }
        L.n_m2l_items = (long long)ib.size();
        // few items (a small tree): share each item's octants among up to 4
        // blocks so that the launch still fills the chip
        // (not with the pair layout, which writes one slot per group)
        L.m2l_split = 1;
        while (!L.m2l_pairs && L.m2l_split < 4 &&
               L.n_m2l_items * 2 * L.m2l_split < M2L_FILL_BLOCKS)
            L.m2l_split *= 2;
        L.m2l_item_ops.alloc(iops.size());
        L.m2l_item_begin.alloc(ib.size());
        L.m2l_item_count.alloc(ib.size());
        L.m2l_item_ops.upload(iops.data(), iops.size(), s);
        L.m2l_item_begin.upload(ib.data(), ib.size(), s);
        L.m2l_item_count.upload(ic.data(), ic.size(), s);
        HIPCHK(hipStreamSynchronize(s));   // host vectors must outlive the copies
    }
    HIPCHK(hipStreamSynchronize(s));
}

}  // namespace afmpb

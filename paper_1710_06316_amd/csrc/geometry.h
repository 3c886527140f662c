// Setup-phase declarations: patch geometry, Morton sort, octree and lists.
#pragma once
#include "common.h"

namespace afmpb {

// Node data in Morton order (structure of arrays).
struct NodeSoA {
    double *x, *y, *z, *nx, *ny, *nz, *area, *rho2;
};

void compute_geometry(const double *V, const int *T, long long n, long long m,
                      double *tri_area, double *tri_n, int *inc_ptr, int *inc_tri,
                      double *area, double *nrm, double *rho2, hipStream_t s);

// centre_third: a root box of 1.5 times the largest extent, with the
// centre of the points' box at 1/3 of it on every axis (false: the tree of
// the matvec, the reference quantisation over the points' own box).
void morton_sort(const double *V, long long n, unsigned long long *keys, int *perm,
                 double lo_out[3], double *scale_out, hipStream_t s, bool centre_third = false);

void gather_nodes(const double *V, const double *nrm, const double *area, const double *rho2,
                  const int *perm, long long n, const NodeSoA &out, hipStream_t s);

// Octree over Morton-sorted keys.  Boxes numbered by ascending (level,
// prefix); level_start[l] is the first box of level l (size nlev + 1).
struct Tree {
    long long nbox = 0;
    int nlev = 0;                      // number of levels present
    std::vector<long long> level_start;
    DBuf<int> level, parent, child_begin, n_child, pt_begin, pt_end;
    DBuf<unsigned long long> prefix;
    DBuf<double> center;               // [nbox][3] physical box centres
    std::vector<double> side;          // physical side length per level
};

void build_tree(const unsigned long long *keys, long long n, int leaf_cap,
                const double lo[3], double scale, Tree &t, hipStream_t s);

// Interaction lists (CSR over boxes, entries ascending).
struct Lists {
    DBuf<int> coll, ncoll;             // [nbox][26] colleagues, count
    DBuf<int> u_ptr, u_idx, v_ptr, v_idx, v_cls, w_ptr, w_idx, x_ptr, x_idx;
    long long n_u = 0, n_v = 0, n_w = 0, n_x = 0;
    // P2P: for each leaf the source boxes U(B) + W(B) + X(A), A = B and its
    // ancestors; work items (leaf, first target point) of <= 64 targets.
    DBuf<int> leaf_ids, p2p_ptr, p2p_src;
    DBuf<int> item_box, item_begin;
    long long n_leaves = 0, n_items = 0, n_p2p_src = 0;
    long long n_p2p_pairs = 0;
    // Balanced P2P work: chunk c = (group, source-range span) with at most
    // P2P_CHUNK source points; group g = (leaf, first of <= 64 targets);
    // chunks of a group are contiguous [grp_ptr[g], grp_ptr[g+1]).
    DBuf<int> ch_lo, ch_hi;              // [n_chunks] range span [lo, hi) in rng
    DBuf<int> rng_b, rng_e;              // [n_rng] source point ranges
    DBuf<int> grp_ptr, grp_tbeg, grp_tend;  // [n_groups+1], [n_groups], [n_groups]
    DBuf<int> ch_grp;                    // [n_chunks] owning group
    long long n_chunks = 0, n_groups = 0, n_rng = 0;
    // Each unordered pair of point sets is evaluated once: a reverse chunk
    // (ch_rev[c] >= 0) also adds the targets' contributions to its sources,
    // stream position k of the chunk going to reverse slot ch_rev[c] + k;
    // ch_rev[c] = -1 for a leaf's own points (one-directional).  The reverse
    // slots of point p are rev_idx[rev_ptr[p] .. rev_ptr[p+1]), in chunk order.
    DBuf<int> ch_rev, rev_ptr, rev_idx;
    long long n_rev = 0;
    // P2M / L2P work: leaves in point order, packed into items of <= 4
    // consecutive leaves with <= 64 points together (a larger leaf alone)
    DBuf<int> pm_leaf, pm_first, pm_count;
    long long n_pm = 0, pm_max_points = 0;
    // the same leaves by decreasing point count (ties in point order): the
    // lane order of the accumulating P2M
    DBuf<int> pm_bysize;
    long long n_pm_leaves = 0;
    DBuf<int> v_tgt;                   // [n_v] target box of each V entry
    // M2L groups: per-entry layout (m2l_grouped = false): group g is V entry g
    // (its source v_idx[g], result slots in list order, [v_ptr[B],
    // v_ptr[B+1]) for target B).  Grouped layout: the V entries of one target
    // that are children of one colleague of its parent, numbered target-major
    // ([vg_ptr[B], vg_ptr[B+1])), vg_src[8 g + c] the child in octant c (-1 if
    // absent).  Items: <= 64 groups of one bucket listed in m2l_cols
    // [m2l_item_begin, + m2l_item_count); m2l_item_ops[8 w + c] is the
    // operator key (level, offset class) of octant slot c, or -1.  Grouped
    // items may share their octants among m2l_split blocks, each with its own
    // result slot per group (slots g * m2l_split + part).
    DBuf<int> vg_ptr, vg_src, m2l_cols;
    DBuf<int> m2l_item_ops, m2l_item_begin, m2l_item_count;
    long long n_vg = 0, n_m2l_items = 0;
    int m2l_split = 1;
    bool m2l_grouped = false;
    // Pair layout (on top of the grouped one): pair q is a box P and one
    // colleague C of it; pr_src[8 q + c] is child c of C (-1 if absent),
    // pr_slot[8 q + b] the grouped-layout slot of (child b of P, C) (-1 if
    // that child has none).  Items: <= 64 pairs of one (level, offset d),
    // pairs [pr_item_begin, + pr_item_count); pr_item_ops[64 w + 8 b + c]
    // the operator key of target octant b and source octant c, or -1.
    bool m2l_pairs = false;
    DBuf<int> pr_src, pr_slot, pr_item_ops, pr_item_begin, pr_item_count;
    long long n_pairs = 0, n_pr_items = 0;
    std::vector<int> levels_with_v;    // levels that have V entries
    // W and X entries by expansions: W entry (B, C) whose point counts have
    // a harmonic mean of at least wx_tau leaves the P2P work; B's points take
    // C's multipole (M2P), C's local expansion takes B's points (P2L).
    // fw_ptr/fw_idx (CSR over boxes): the far W boxes of each leaf;
    // m2p_leaf/m2p_tb: one item per 64 points of such a leaf; fx_ptr/fx_idx:
    // the far X leaves of each box; p2l_box: the boxes that have any.
    int wx_tau = 0;
    DBuf<int> fw_ptr, fw_idx, m2p_leaf, m2p_tb, fx_ptr, fx_idx, p2l_box;
    long long n_wx_far = 0, n_wx_pairs = 0, n_m2p_items = 0, n_p2l_boxes = 0;
};

// M2L layout: 1 per entry, 2 grouped, 3 pairs (with the grouped slots), 0
// chosen by the number of V entries (pairs only where auto_pairs).
// p2p_chunks = false leaves out the matvec's symmetric P2P work (chunks and
// reverse slots); the per-leaf source box lists are built either way.
// wx_tau > 0 (with p2p_chunks) moves the W/X entries of harmonic-mean point
// count >= wx_tau to expansions.
void build_lists(const Tree &t, Lists &L, int m2l_layout, hipStream_t s,
                 bool p2p_chunks = true, bool auto_pairs = true, int wx_tau = 0);

}  // namespace afmpb

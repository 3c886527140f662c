// Right-hand side of Eq. (5) and the reaction potential at the atoms by a
// fast multipole pass over disjoint source and target sets (Section 2:
// the right-hand side is itself an FMM evaluation; Section 3.3: trees of
// separate source and target points).  One octree holds the nodes and the
// atoms together (one Morton quantisation of their common bounding box);
// every box knows its range of nodes and its range of atoms, each set in its
// own Morton order.
//   right-hand side: atom charges q/eps_s -> potential and normal derivative
//                    at the nodes;
//   energy:          node charges a h and dipoles -a f / ebar along the node
//                    normals -> Laplace potential at the atoms, times ebar.
#pragma once
#include "fmm.h"

namespace afmpb {

struct DualTree {
    bool built = false;
    long long n = 0, na = 0;
    Tree t;
    Lists L;
    Fmm F;
    double lo[3] = {0, 0, 0}, scale = 1;
    DBuf<int> node_main;                 // [n] dual node position -> Morton position
    DBuf<int> atom_caller;               // [na] dual atom position -> caller index
    DBuf<int> nptb, npte, aptb, apte;    // [nbox] node / atom range of each box
    DBuf<int> npm_leaf, npm_first, npm_count, apm_leaf, apm_first, apm_count;
    DBuf<int> npm_bysize, apm_bysize;    // item leaves by decreasing point count
    long long n_npm_leaves = 0, n_apm_leaves = 0;
    long long n_npm = 0, npm_max = 0, n_apm = 0, apm_max = 0;
    DBuf<double> nodes;                  // [6][n] x y z nx ny nz, dual node order
    DBuf<double> atoms;                  // [6][na] x y z and zero normals
    DBuf<double> aq;                     // [na] charges, dual atom order
    DBuf<double> zero;                   // [max(n, na)] zeros (no dipoles)
    DBuf<double> srcf, srch;             // [max(n, na)] source strengths
    // P2P groups of <= 64 targets of one leaf: leaf position, target range
    DBuf<int> gn_leaf, gn_b, gn_e;       // node targets (right-hand side)
    DBuf<int> ga_leaf, ga_b, ga_e;       // atom targets (energy)
    long long n_gn = 0, n_ga = 0;
    DBuf<double> far;
    FarWork<double> w{};
    DBuf<double> pv, pdv;                // P2P potential / normal derivative
    DBuf<double> dscratch;               // reduction partials (sized at setup)
};

}  // namespace afmpb

// Far field of the matvec: expansions, translation operators and the
// P2M / M2M / M2L / L2L / L2P passes.
#pragma once
#include "geometry.h"

namespace afmpb {

constexpr int MAXP = 20;

// Device-side view of the per-level basis constants.
struct BasisDev {
    int P, K;
    int screened;              // 1: kernel 1 is e^{-kappa r}/(4 pi r); 0: both Laplace
    double kappa;
    const double *norm;        // [K]
    const double *inv_dfact;   // [P+2]   1/(2n+1)!!
    const double *ginv;        // [nlev][P+1]  1/g_n(kappa s_l)
    const double *side;        // [nlev]
    const double *rec;         // [P+1][P+1][2] recurrence coefficients of the harmonics
    const double *gser;        // [2][GSER] term ratios of the g_n series (n = P, P-1)
};

struct Fmm {
    int P = 0, K = 0, nlev = 0;
    double kappa = 0;
    int screened = 0;
    long long nkey = 0;                  // (nlev-2)*316 translation classes
    DBuf<double> norm, inv_dfact, ginv, kinv, weight, side, rec, gser;
    DBuf<double> T;                      // [2][nkey][K][K] M2L, row = local index
    DBuf<double> Ut;                     // [2][nlev][8][K][K] transposed M2M operator
    // Operators in matrix-core operand order: per matrix [K/16 row tiles]
    // [KK/4 k-steps][64 lanes], lane l holding A[16 rt + l%16][4 ks + l/16]
    // (zero padded); PM elements per matrix.
    long long PM = 0;
    int KK = 0;
    int KZ = 0;                          // M2L result slot length: K rounded up to 16
    DBuf<double> Tp, Up, Lp;             // M2L, M2M (A = U), L2L (A = U^T)
    DBuf<float> Tp32, Up32, Lp32;
    // M2L operators split into bf16 high and low parts, in the operand order
    // of the 16x16x32 bf16 matrix instruction: per matrix [K/16 row tiles]
    // [KC = ceil(K/32) k-chunks][64 lanes][8], lane l holding
    // A[16 rt + l%16][32 kc + 8 (l/16) + e] (zero padded); PMB per matrix
    int KC = 0;
    long long PMB = 0;
    DBuf<unsigned short> Tbh, Tbl;
    BasisDev dev() const {
        return BasisDev{P, K, screened, kappa, norm.p, inv_dfact.p, ginv.p, side.p, rec.p, gser.p};
    }
};

void build_fmm_operators(const Tree &t, const Lists &L, int P, double kappa, bool bf16_m2l,
                         Fmm &F, hipStream_t s);

// Far-field evaluation for one matvec.  sf = a*f, sh = a*h per node (Morton
// order).  Writes phi[4][n] = {Phi_L, dPhi_L/dn, Phi_Y, dPhi_Y/dn} at every
// node (zero where no local expansion exists).
template <typename R>
struct FarWork {
    R *M, *Lc, *Z, *phi;       // [nbox][2][K], [nbox][2][K], [n_v][2][KZ], [4][n]
    R *Mt;                     // [8][widest level][2][K] per-octant M2M products
    int bf16_m2l = 0;          // FP32 path: M2L as three bf16 products (split operands)
    hipEvent_t p2m_done = nullptr;   // recorded once the multipole expansions are formed
};

template <typename R>
void far_field(const Fmm &F, const Tree &t, const Lists &L, const NodeSoA &nd,
               const R *px, const R *py, const R *pz, const R *pnx, const R *pny,
               const R *pnz, const R *sf, const R *sh, double inv_ebar, long long n,
               const FarWork<R> &w, struct Prof *prof, hipStream_t s);

// One side (sources or targets) of a far-field pass over a tree whose boxes
// may hold two point sets: per box the range [ptb[b], pte[b]) of this side's
// points (in this side's own order), the P2M / L2P items over the leaves
// that hold points of this side, and the points (positions, unit normals).
template <typename R>
struct FarSide {
    const int *ptb = nullptr, *pte = nullptr;
    const int *pm_leaf = nullptr, *pm_first = nullptr, *pm_count = nullptr;
    long long n_pm = 0, pm_max_points = 0;
    const int *pm_bysize = nullptr;   // the item leaves by decreasing point count
    long long n_pm_leaves = 0;
    const R *x = nullptr, *y = nullptr, *z = nullptr, *nx = nullptr, *ny = nullptr,
            *nz = nullptr;
    long long n = 0;
};

// Far field from the sources of `src` (charge sh, dipole -sf along the
// source normal; the dipoles of kernel 0 scaled by inv_ebar) to the targets
// of `dst`: phi[4][dst.n] as far_field.  Leaves without source points are
// left out of src's items, so their multipoles are cleared first.
template <typename R>
void far_field_sides(const Fmm &F, const Tree &t, const Lists &L, const FarSide<R> &src,
                     const R *sf, const R *sh, const FarSide<R> &dst, double inv_ebar,
                     const FarWork<R> &w, struct Prof *prof, hipStream_t s);

}  // namespace afmpb

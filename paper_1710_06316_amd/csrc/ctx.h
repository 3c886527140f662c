// Internal: the solver context behind the C ABI, and the setup / solve
// routines that the context entry points and the solve server share.
#pragma once
#include <algorithm>
#include <cmath>
#include <string>

#include "../../include/afmpb.h"
#include "dual.h"
#include "gmres.h"
#include "krylov.h"
#include "matvec.h"
#include "prof.h"

using namespace afmpb;

struct afmpb_ctx {
    // caller's device memory supplier (first member: the buffers below refer
    // to it until they are freed)
    afmpb_allocator al{};
    bool has_al = false;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;  // created by the context (NULL stream given)
    // second stream for the near field, forked from and joined to `stream`
    // inside every matvec (default priority)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_p2m = nullptr;
    std::string err;
    bool loaded = false;
    afmpb_params prm{};
    long long n = 0, m = 0, na = 0;
    double ebar = 1, alpha = 1, inv_ebar = 1;
    double ms_setup = 0;
    double ms_phase[AFMPB_SETUP_PHASES] = {};   // setup wall time per phase
    DBuf<double> V, ax, aq, tri_area, tri_n, area_c, nrm_c, rho2_c;
    DBuf<int> T, inc_ptr, inc_tri, perm;
    DBuf<unsigned long long> keys;
    DBuf<double> node64;      // 8n: x y z nx ny nz area rho2
    DBuf<float> node32;       // 6n
    double lo[3] = {0, 0, 0}, scale = 1;
    Tree tree;
    Lists lists;
    NearSet near;
    Fmm fmm;
    DualTree dual;            // nodes + atoms tree of the FMM right-hand side
    DBuf<double> w64, far64, p2p64, p2p_part, p2p_rpart;
    DBuf<float> w32, far32;
    MatvecPlan<double> mp64;
    MatvecPlan<float> mp32;
    // vectors in Morton order
    DBuf<double> xa, ya, bvec, xsol, tmp, hbuf, dscratch, phi_at, dotv;
    DBuf<double> krylov;
    int krylov_m = 0;
    Prof prof;
    // device address of the static scratch of the allocation-free energy
    // entry point on this context's device (resolved at creation)
    double *noalloc_part = nullptr;
    // GMRES on the device (state, captured Arnoldi steps); declared last so
    // that its graphs go before the buffers they use
    GmresEngine gm;

    NodeSoA nodes() const {
        double *b = node64.p;
        long long N = n;
        return NodeSoA{b, b + N, b + 2 * N, b + 3 * N, b + 4 * N, b + 5 * N, b + 6 * N, b + 7 * N};
    }
    void sync() { HIPCHK(hipStreamSynchronize(stream)); }
    void matvec_m(const double *x, double *y, bool fp64) {
        if (fp64 || prm.precision == AFMPB_FP64) apply_operator<double>(mp64, x, y, &prof, stream);
        else apply_operator<float>(mp32, x, y, &prof, stream);
    }
};

namespace afmpb {

// 4 pi times the Coulomb constant in kcal A / (mol e^2): internal units of
// the potentials -> kcal/(mol e)
double unit_scale();
void fill_defaults(afmpb_params &p);
// validated copy of the caller's parameters (zeros -> defaults)
afmpb_params normalise(const afmpb_params &in);
// geometry, keys, tree, lists, near set, operators and matvec plans
void load_molecule(afmpb_ctx *c, long long n, const double *xyz, long long m, const int *tri,
                   long long na, const double *axyz, const double *q, const afmpb_params &prm);
// polar energy (kcal/mol) of the solution x (Morton order, internal units);
// synchronises the context stream
double energy_of(afmpb_ctx *ctx, const double *x_morton);
// right-hand side / energy by the fast multipole pass over nodes and atoms
// (dual.hip): whether the context uses it, its setup, b (Morton order) and
// the device scalar sum_k q_k phi_reac(r_k)
bool use_dual(const afmpb_ctx *c);
void build_dual(afmpb_ctx *c);
void dual_rhs(afmpb_ctx *c, double *b_morton);
void dual_energy_sum(afmpb_ctx *c, const double *x_morton, double *out);
// enqueue on the context stream, by the direct sums or the FMM pass: the
// right-hand side (Morton order) and the device scalar sum_k q_k phi_reac
void rhs_morton(afmpb_ctx *c, double *b_morton);
void energy_sum(afmpb_ctx *c, const double *x_morton, double *out);
// device address of the allocation-free entry point's static scratch on
// `device` (looked up once per device); the energy from caller-order x on
// the device into a device scalar, with no allocation and no synchronisation
double *noalloc_scratch(int device);
void energy_noalloc(afmpb_ctx *c, const double *x_dev, double *energy_dev);

}  // namespace afmpb

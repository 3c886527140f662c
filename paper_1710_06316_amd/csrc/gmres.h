// Restarted GMRES with the Arnoldi process, the Givens least-squares update
// and the stopping test (Section 3.4, Eq. 7) held on the GPU: one Arnoldi
// step is a fixed sequence of kernels that read the step index and the
// convergence flag from device memory, so it is captured once into a HIP
// graph and replayed; the host only reads a small status block per step.
#pragma once
#include "common.h"

struct afmpb_ctx;

namespace afmpb {

// Device-resident state of one GMRES cycle (copied to the host after a step).
struct GmresState {
    int j;            // Arnoldi steps (columns of H) taken in this cycle
    int done;         // the cycle has ended: converged, breakdown or m steps
    int converged;    // the residual estimate met the tolerance (or breakdown)
    int active;       // the last step changed the state (0: it found done set)
    int steps;        // Arnoldi steps over all cycles
    int pad[3];
    double tol;       // rel_tol ||b|| + abs_tol of the current run
    double beta;      // residual norm at the start of the cycle
    double est;       // |g_{j}|: residual estimate after the last step
    double hn;        // norm of the last orthogonalised vector
    double inv;       // 1/hn (or 1/beta at the cycle start)
    double pad2[3];
};

struct GmresEngine {
    int m = 0;
    long long len = 0;
    long long nblk = 0;                       // vector chunks of the reductions
    DBuf<GmresState> st;                      // [1]
    DBuf<double> H;                           // [m][m+1], column j contiguous
    DBuf<double> cs, sn, g, y, h1, h2, part;  // part: [m+1][nblk] partial sums
    GmresState *host = nullptr;               // pinned: [3] status slots
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipGraphExec_t step_exec[2] = {nullptr, nullptr};   // [fp64, fp32]
    hipGraph_t step_graph[2] = {nullptr, nullptr};
    ~GmresEngine();
    void reset();
};

struct GmresResult {
    int iterations = 0, restarts = 0;
    long long inner = 0;
    double est = 0, true_rel = 0;
    bool converged = false;
};

// Restarted GMRES(m) on M x = b (Morton order, device vectors of the
// context); x_zero starts from x = 0.  The operator is the FP64 or FP32
// matvec.  final_residual: recompute ||b - M x|| with the FP64 operator.
GmresResult gmres_device(afmpb_ctx *c, const double *b, double *x, bool x_zero, double rel_tol,
                         double abs_tol, int m, int max_restarts, bool fp64,
                         bool final_residual);

// Pieces for an asynchronous driver (the solve server), all enqueued on the
// context stream: prepare the engine for restart m (allocations and graph
// captures; not under another capture), start a cycle from r0 = b - M x (or
// b when x_first_zero), one Arnoldi step (graph launch and status copy into
// host slot `slot`), and the end of a cycle (x += V y).
void gmres_prepare(afmpb_ctx *c, int m, bool need_fp32);
void gmres_set_tol(afmpb_ctx *c, const double *b, double rel_tol, double abs_tol, int slot);
void gmres_cycle_start(afmpb_ctx *c, const double *b, const double *x, bool x_first_zero,
                       bool fp64, int slot);
void gmres_step(afmpb_ctx *c, bool fp64, int slot);
void gmres_cycle_end(afmpb_ctx *c, double *x);
const GmresState &gmres_status(afmpb_ctx *c, int slot);

}  // namespace afmpb

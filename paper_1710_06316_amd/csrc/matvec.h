// The per-iteration operator y = M x of Eq. (5), assembled from the far
// field (fmm.hip), P2P, the near-set corrections and the identity term.
#pragma once
#include "fmm.h"
#include "near.h"

namespace afmpb {

template <typename R>
struct NodeR {
    const R *x, *y, *z, *nx, *ny, *nz;
};

// From this many nodes on, the automatic schedule runs every kernel on one
// stream: the kernels are then large enough to fill the GPU alone, and run
// beside each other they compete for the same SIMDs and caches (measured on
// the 9.7M-node shell: 67.1 ms one stream, 68.1-68.4 ms with either
// two-stream order).
constexpr long long SERIAL_MIN_NODES = 1ll << 20;

template <typename R>
struct MatvecPlan {
    long long n = 0;
    const Tree *tree = nullptr;
    const Lists *lists = nullptr;
    const Fmm *fmm = nullptr;
    const NearSet *near = nullptr;
    NodeSoA nd64{};            // double node data (Morton order)
    NodeR<R> nd{};             // node data in the working precision
    const double *area = nullptr;
    double kappa = 0, inv_ebar = 0, alpha = 0;
    R *sf = nullptr, *sh = nullptr;
    R *xp = nullptr;                       // [n][2] (f, h) in the working precision
    double *pf = nullptr, *ph = nullptr;   // P2P sums (double in both precisions)
    double *part = nullptr;                // P2P chunk partial sums [chunks][2][64]
    double *rpart = nullptr;               // P2P reverse partial sums [reverse slots][2]
    const R *delta = nullptr;              // near corrections [nnz][4], working precision
    hipStream_t side = nullptr;            // near field runs here, between fork and join
    hipEvent_t fork = nullptr, join = nullptr;
    // P2P waits for P2M (far.p2m_done); the near correction runs first
    bool late_p2p = false;
    bool serial = false;                   // no second stream: every kernel on s
    FarWork<R> far{};
};

// x, y: [2n] in Morton order, double.  y must not alias x.
template <typename R>
void apply_operator(const MatvecPlan<R> &mp, const double *x, double *y, Prof *prof,
                    hipStream_t s);

void to_morton(const double *in, const int *perm, long long n, double *out, hipStream_t s);
void from_morton(const double *in, const int *perm, long long n, double *out, hipStream_t s);

}  // namespace afmpb

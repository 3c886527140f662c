/*
 * afmpb.h -- C ABI of the MI355X node-patch Poisson-Boltzmann solver.
 *
 * The library applies and solves the boundary-integral system of the
 * linearised Poisson-Boltzmann equation as discretised by the node-patch
 * scheme (Zhang et al., Section 2):
 *
 *   [ alpha I + B    -A        ] [f]   1     [ sum_k q_k G_pk       ]
 *   [ D              alpha I - C] [h] = ---- [ sum_k q_k dG_pk/dn_0 ]   (Eq. 5)
 *                                      eps_s
 *
 * with alpha = 1/(2 ebar) + 1/2, ebar = eps_s/eps_p, and A, B, C, D the patch
 * integrals of Eq. (6).  Far pairs use the integrand at the node times the
 * patch area; pairs within the near set N(p) = {p} U {t : |x_p-x_t| <
 * eta max(rho_p, rho_t)} (rho = patch radius) use the patch integrals.  The
 * point-rule sums run through an adaptive fast multipole method (Laplace and
 * screened-Coulomb kernels, P2P near field, P2M/M2M/M2L/L2L/L2P far field).
 *
 * Conventions
 *  - Every function returns afmpb_status: 0 on success, < 0 on error.  No
 *    C++ exception crosses the ABI.  afmpb_last_error() gives the message of
 *    the last failing call on a context.
 *  - Ownership: the caller owns every array it passes.  afmpb_set_molecule
 *    copies its inputs before returning; the context owns all device state
 *    (tree, lists, near coefficients, expansions, Krylov basis) until
 *    afmpb_destroy or the next afmpb_set_molecule.
 *  - Pointers are host pointers unless the name ends in _dev; _dev pointers
 *    are device pointers on the context's device, used in order on the
 *    context's stream.
 *  - Node order in every input/output array is the caller's order (the
 *    Morton permutation is internal).  Vectors are x = [f(0..N-1); h(0..N-1)].
 *  - Units: coordinates in Angstrom, charges in e, kappa in 1/Angstrom.  The
 *    matvec is unitless.  afmpb_solve returns f in kcal/(mol e), h in
 *    kcal/(mol e A) and the energy in kcal/mol.
 *  - A context is used by one host thread at a time.
 *  - After any error other than AFMPB_E_DEVICE the context stays usable
 *    (a failed afmpb_set_molecule leaves it with no molecule).
 */
#ifndef AFMPB_H
#define AFMPB_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AFMPB_OK = 0,
    AFMPB_E_INVALID = -1,        /* bad argument (NULL, size, NaN, eps<=0, kappa<0 ...) */
    AFMPB_E_MESH = -2,           /* mesh not closed, non-manifold, duplicate vertex,
                                    degenerate triangle or inward orientation        */
    AFMPB_E_OOM = -3,            /* device allocation failed; nothing half-built kept */
    AFMPB_E_NOT_CONVERGED = -4,  /* solve: outputs hold the last iterate, info filled */
    AFMPB_E_NUMERIC = -5,        /* NaN/Inf met in an iterate or input vector          */
    AFMPB_E_DEVICE = -6,         /* HIP runtime error; the context must be destroyed   */
    AFMPB_E_STATE = -7,          /* call out of order (e.g. matvec before a molecule)  */
    AFMPB_E_PENDING = -8,        /* server: request not finished yet                   */
    AFMPB_E_CANCELLED = -9       /* server: request cancelled                          */
} afmpb_status;

typedef enum {
    AFMPB_FP64 = 0,              /* every kernel in double precision                   */
    AFMPB_FP32_REFINED = 1,      /* FMM translations and P2P pair terms in single
                                    precision; P2P sums each 64-source tile in single
                                    and adds a target's tiles in double; near
                                    corrections stored in single, applied in double;
                                    Arnoldi, residuals and energy in double; iterative
                                    refinement restores the residual               */
    AFMPB_FP32_BF16M2L_REFINED = 2 /* as AFMPB_FP32_REFINED, with the M2L products taken
                                    as three bf16 products of split operands (hi*hi +
                                    hi*lo + lo*hi, FP32 accumulation) on the bf16
                                    matrix instruction; about 2^-16 relative error per
                                    product, which the refinement loop absorbs      */
} afmpb_precision;

/* Problem and solver parameters (the problem statement of Section 2 and the
 * GMRES settings of Sections 3.4 and 5). */
typedef struct {
    double eps_p;        /* interior dielectric constant (> 0)                      */
    double eps_s;        /* exterior (solvent) dielectric constant (> 0)            */
    double kappa;        /* Debye-Hueckel parameter, 1/A (>= 0; 0 = no salt)        */
    int order_p;         /* multipole expansion order p (2..20); 0 selects 8        */
    int leaf_cap;        /* max nodes per leaf box (>= 1); 0 selects 64;  a value
                            >= N makes the root a leaf: every pair by direct P2P   */
    int precision;       /* afmpb_precision                                         */
    double rel_tol;      /* GMRES stops at ||r|| <= rel_tol ||b||_2 + abs_tol (Eq. 7) */
    double abs_tol;
    int restart;         /* Krylov vectors per GMRES cycle (>= 1); 0 selects 80     */
    int max_restarts;    /* restarts after the first cycle (>= 0)                   */
    double near_eta;     /* near-set radius factor eta (> 0); 0 selects 4           */
    int m2l_layout;      /* M2L work layout: 0 automatic; 1 one result slot per
                            V-list entry, items of one (level, offset class);
                            2 one slot per (target, colleague of its parent),
                            all children of the colleague accumulated in
                            registers; 3 as 2, with work items of box pairs
                            (P, colleague C of P): each child of C is read
                            once for all children of P.  Automatic takes 2
                            from 2^21 V-list entries on (large trees, where
                            the result traffic of 1 dominates) and 3 from
                            2^23.  Every layout computes the same sums
                            (rounding order aside; 2 and 3 bit for bit)       */
    int rhs_fmm;         /* right-hand side of Eq. (5) and the reaction potential
                            at the atoms: 0 automatic (fast multipole pass over
                            one octree of nodes and atoms from 2^34 node-atom
                            pairs on, direct sums below); 1 direct sums; 2 the
                            fast multipole pass (order max(order_p, 14), FP64) */
    int overlap;         /* near-field schedule inside a matvec, beside the
                            far-field chain on a second stream: 0 automatic
                            (3 from 2^20 nodes on, else 1); 1 P2P, then the
                            near-set correction, both started with the chain;
                            2 the near-set correction beside P2M, then P2P
                            after P2M has finished (beside the translations);
                            3 one stream, every kernel after the last (for
                            per-kernel timing).  All give bit-identical
                            products                                           */
    int wx_expand;       /* W and X lists (Section 3.2): 0 automatic (direct
                            P2P: on the trees measured, P2P's cost per pair is
                            below that of the expansions it would replace);
                            1 every W/X point pair by direct P2P; n >= 2 (order_p
                            6, 8, 10 or 14) a W entry (leaf B, box C) whose
                            point counts have a harmonic mean
                            2|B||C|/(|B|+|C|) >= n is taken by expansions:
                            C's multipole evaluated at B's points (M2P) and
                            B's points added to C's local expansion (P2L);
                            the others stay in P2P.  Truncation error of the
                            same order as the M2L's                          */
} afmpb_params;

typedef struct {
    int iterations;              /* Arnoldi steps (matrix-vector products in GMRES) */
    int restarts;
    long long inner_products;    /* dot products and norms taken by the Arnoldi process */
    double rel_residual_estimate;/* GMRES estimate / ||b|| at exit                    */
    double true_rel_residual;    /* ||b - M x|| / ||b|| recomputed in FP64 at exit    */
    int converged;
    int refinement_steps;        /* outer refinement steps (FP32_REFINED only)        */
    double ms_setup;             /* last afmpb_set_molecule: geometry, tree, lists,
                                    near coefficients, translation operators          */
    double ms_rhs, ms_gmres, ms_energy, ms_total;
} afmpb_solve_info;

/* Sizes of the internal tree, for afmpb_debug_tree. */
typedef struct {
    long long n_nodes, n_boxes, n_levels;
    long long n_u, n_v, n_w, n_x;    /* entries of the U, V, W, X lists         */
    long long n_near;                /* entries of the near set (incl. diagonal)*/
    long long n_p2p_pairs;           /* point pairs evaluated by P2P per matvec  */
    long long n_m2l_pairs;           /* V-list box pairs per matvec              */
    int order_p, leaf_cap;
    long long n_m2l_slots;           /* M2L result slots per kernel and matvec
                                        (= n_m2l_pairs in the per-entry layout)  */
    int m2l_layout;                  /* layout in use: 1 per entry, 2 grouped,
                                        3 pairs                              */
    int rhs_mode;                    /* right-hand side / energy: 1 direct sums,
                                        2 fast multipole pass over nodes+atoms */
    long long rhs_boxes;             /* boxes of the nodes+atoms tree (0 if 1) */
    long long n_wx_far;              /* W entries taken by expansions (M2P+P2L) */
    long long n_wx_pairs;            /* point pairs they stand for (n_p2p_pairs
                                        excludes them)                        */
} afmpb_tree_sizes;

/* Caller-allocated host buffers for afmpb_debug_tree (sizes from
 * afmpb_tree_info).  Any pointer may be NULL to skip that array.  Boxes are
 * numbered by ascending (level, prefix); lists are CSR over boxes with
 * entries ascending; point indices are positions in Morton order. */
typedef struct {
    unsigned long long *keys;        /* [n_nodes] sorted 63-bit Morton keys      */
    int *perm;                       /* [n_nodes] Morton position -> caller index */
    int *level, *parent, *child_begin, *n_child, *pt_begin, *pt_end;  /* [n_boxes] */
    unsigned long long *prefix;      /* [n_boxes]                                 */
    int *u_ptr, *u_idx;              /* [n_boxes+1], [n_u]                        */
    int *v_ptr, *v_idx, *v_class;    /* [n_boxes+1], [n_v], [n_v] (0..315)        */
    int *w_ptr, *w_idx;              /* [n_boxes+1], [n_w]                        */
    int *x_ptr, *x_idx;              /* [n_boxes+1], [n_x]                        */
    long long *near_ptr;             /* [n_nodes+1]                               */
    int *near_col;                   /* [n_near]                                  */
    double *near_delta;              /* [n_near][4]: patch minus point-rule value
                                        of {A,B,C,D} (point value 0 on the diagonal) */
} afmpb_tree_view;

typedef struct afmpb_ctx afmpb_ctx;

/* Device memory supplier for a context (e.g. a framework's caching
 * allocator).  alloc returns `bytes` of device memory on the context's
 * device, usable by work queued on `stream` (the context's stream), or NULL
 * when it cannot; free returns memory alloc gave.  The library waits for its
 * own queued work before it frees.  Both are called from the thread that
 * makes the library call; user is passed through. */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *user);
    void (*free)(void *ptr, void *user);
    void *user;
} afmpb_allocator;

/* Fills *out with the defaults above (eps_p 2, eps_s 80, kappa 0.1, p 8,
 * leaf 64, FP64, rel_tol 1e-6, abs_tol 0, restart 80, max_restarts 5,
 * eta 4, automatic right-hand side and schedule). */
afmpb_status afmpb_default_params(afmpb_params *out);

/* Creates a context on HIP device `device`.  hip_stream is a hipStream_t on
 * which all work of this context is queued; it must outlive the context.
 * NULL: the context creates a non-blocking stream of its own (the solve
 * captures its Arnoldi steps into HIP graphs, which the legacy null stream
 * does not allow); the _dev entry points then order against other work only
 * through device synchronisation.  alloc (may be NULL: hipMalloc / hipFree)
 * supplies every device buffer of the context (tree, lists, near set,
 * operators, expansions, Krylov basis, work vectors); the struct is copied.
 * Errors: AFMPB_E_INVALID (no such device, NULL out, incomplete allocator),
 * AFMPB_E_DEVICE. */
afmpb_status afmpb_create(int device, void *hip_stream, const afmpb_allocator *alloc,
                          afmpb_ctx **out);

/* Frees all device state of the context.  NULL is accepted. */
afmpb_status afmpb_destroy(afmpb_ctx *ctx);

/* Message of the last failing call on ctx ("" if none).  Valid until the
 * next call on ctx. */
const char *afmpb_last_error(const afmpb_ctx *ctx);

/* Loads a molecule and builds everything that does not depend on the
 * unknowns (Section 2 computation flow, steps 1-2; the phased tree/DAG
 * construction of Section 3.3): validates the mesh, uploads it, computes
 * patch geometry, Morton keys and the adaptive octree, the U/V/W/X lists,
 * the near set with its patch-integral corrections, and the translation
 * operators.  xyz: [n_nodes][3] node coordinates.  tri: [n_tri][3] 0-based
 * node indices, counter-clockwise seen from the solvent (outward normal).
 * atom_xyz [n_atoms][3], charge [n_atoms]; radius [n_atoms] may be NULL (not
 * used by the solver).  Errors: AFMPB_E_INVALID, AFMPB_E_MESH, AFMPB_E_OOM,
 * AFMPB_E_DEVICE. */
afmpb_status afmpb_set_molecule(afmpb_ctx *ctx, long long n_nodes,
                                const double *xyz, long long n_tri,
                                const int *tri, long long n_atoms,
                                const double *atom_xyz, const double *charge,
                                const double *radius,
                                const afmpb_params *params);

/* y = M x for the left-hand side operator of Eq. (5), one FMM evaluation
 * (the per-iteration matrix-vector product of Section 2, step 3).
 * x, y: [2 n_nodes] host arrays, caller order.  Uses the precision chosen in
 * the parameters.  Errors: AFMPB_E_STATE (no molecule), AFMPB_E_NUMERIC
 * (non-finite x), AFMPB_E_DEVICE. */
afmpb_status afmpb_matvec(afmpb_ctx *ctx, const double *x, double *y);

/* As afmpb_matvec with device pointers, enqueued on the context's stream
 * without host synchronisation.  x_dev and y_dev must not overlap.  No
 * finiteness check. */
afmpb_status afmpb_matvec_dev(afmpb_ctx *ctx, const double *x_dev,
                              double *y_dev);

/* Solves Eq. (5) by restarted GMRES (Section 3.4; stopping rule Eq. 7) and
 * evaluates the polar energy 1/2 sum_k q_k phi_reac(r_k), phi_reac from the
 * interior Green representation on the surface.  x0: optional warm start
 * [2 n_nodes] in internal (unitless) form as returned by a previous solve
 * divided by the unit factor, or NULL for zero.  f, h: [n_nodes] outputs
 * (may be NULL); energy: scalar output (may be NULL); info may be NULL.
 * On AFMPB_E_NOT_CONVERGED the outputs hold the last iterate. */
afmpb_status afmpb_solve(afmpb_ctx *ctx, const double *x0, double *f,
                         double *h, double *energy, afmpb_solve_info *info);

/* Right-hand side of Eq. (5) in caller order ([2 n_nodes], unitless). */
afmpb_status afmpb_rhs(afmpb_ctx *ctx, double *b);

/* Switches the working precision of the loaded molecule between AFMPB_FP64
 * and AFMPB_FP32_REFINED (both operator forms are built by
 * afmpb_set_molecule); AFMPB_FP32_BF16M2L_REFINED only if the molecule was
 * set up with it (its split operators are built then).  Applies to later
 * matvec and solve calls.  Errors: AFMPB_E_STATE (no molecule),
 * AFMPB_E_INVALID. */
afmpb_status afmpb_set_precision(afmpb_ctx *ctx, int precision);

/* Polar energy (kcal/mol) for a given internal solution x = [f; h]
 * (caller order, unitless). */
afmpb_status afmpb_energy(afmpb_ctx *ctx, const double *x, double *energy);

/* Allocation-free form of afmpb_energy, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops).
 * x_dev: [2 n_nodes] device array, caller order, internal (unitless) units;
 * energy_dev: one device double receiving the polar energy (kcal/mol).  Both
 * on the context's device; the work is enqueued on the context's stream with
 * no allocation, free or host synchronisation.  Its only scratch is a fixed
 * device array of 16,384 doubles (one partial sum per block of 256 atoms),
 * which each GPU holds until the process ends and which every call on that
 * GPU shares: calls that overlap on one GPU (other streams, other contexts)
 * race on it.  Each call writes every partial it reads, so nothing needs
 * clearing.  Errors: AFMPB_E_INVALID (null pointer, or more than 4,194,304
 * atoms), AFMPB_E_STATE (no molecule), AFMPB_E_DEVICE. */
afmpb_status afmpb_energy_dev_noalloc(afmpb_ctx *ctx, const double *x_dev,
                                      double *energy_dev);

/* Wall time (ms) of the phases of the last afmpb_set_molecule: 0
 * validation, upload and patch geometry; 1 Morton keys, sort and node
 * gather; 2 octree; 3 U/V/W/X lists and the P2P / M2L work items; 4 near
 * set (the patch-integral corrections are then computed on a second stream
 * while phases 2, 3, 5, 6 and 7 run); 5 translation operators; 6 work
 * buffers and structural checks; 7 the octree of nodes and atoms for the
 * fast multipole right-hand side and energy (empty when direct sums are
 * used); 8 the wait for the patch-integral corrections after all the rest.
 * Run order: 0, 1, 4, 2, 3, 5, 6, 7, 8.
 * ms: [AFMPB_SETUP_PHASES] host array. */
#define AFMPB_SETUP_PHASES 9
afmpb_status afmpb_setup_times(afmpb_ctx *ctx, double *ms);

/* Sizes of the internal tree and lists of the loaded molecule. */
afmpb_status afmpb_tree_info(afmpb_ctx *ctx, afmpb_tree_sizes *out);

/* Copies the internal tree, lists and near set to caller buffers. */
afmpb_status afmpb_debug_tree(afmpb_ctx *ctx, const afmpb_tree_view *out);

/* Per-kernel timing with HIP events on the context's stream.  enable != 0
 * starts recording (and clears the totals); 0 stops.  afmpb_profile_read
 * returns, for entry idx (0-based), its name, total milliseconds and launch
 * count; AFMPB_E_INVALID past the last entry.  Names stay valid until the
 * context is destroyed. */
afmpb_status afmpb_profile_enable(afmpb_ctx *ctx, int enable);
afmpb_status afmpb_profile_read(afmpb_ctx *ctx, int idx, const char **name,
                                double *total_ms, long long *launches);
/* Restricts the timing to the scopes named `scope` (a name afmpb_profile_read
 * reports, e.g. "m2l"); NULL or "" times every scope again.  Each timed scope
 * costs two event records on its stream, so timing one kernel perturbs the
 * matvec far less than timing all of them.  The string is copied. */
afmpb_status afmpb_profile_only(afmpb_ctx *ctx, const char *scope);

/* ------------------------------------------------------------------------
 * Solve server: continuous batching of independent solves on one device.
 *
 * Requests are admitted in arrival order while the device bytes of the
 * admitted molecules stay within hbm_budget_bytes (a single request larger
 * than the budget runs alone) and fewer than max_active are in flight.  Each
 * admitted molecule gets its own context and stream; its matvec is captured
 * once into HIP graphs, and one host thread advances all admitted solves by
 * one asynchronous GMRES chunk (one Arnoldi step) at a time, so their work
 * overlaps on the device and late arrivals join while others run.  Every
 * solve follows the same algorithm, kernels and order as afmpb_solve on the
 * same molecule and parameters, so its result does not depend on what else
 * is in flight.  All server functions are thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct afmpb_server afmpb_server;

/* One request: host arrays as for afmpb_set_molecule (copied on submit). */
typedef struct {
    long long n_nodes;
    const double *xyz;            /* [n_nodes][3]                           */
    long long n_tri;
    const int *tri;               /* [n_tri][3], outward (solvent) orientation */
    long long n_atoms;
    const double *atom_xyz;       /* [n_atoms][3]                           */
    const double *charge;         /* [n_atoms]                              */
} afmpb_molecule;

/* Per-size choice of leaf capacity and expansion order, used for requests
 * when the server's parameters have leaf_cap == 0 or order_p == 0: the first
 * entry with n_nodes <= max_nodes applies (entries ascending in max_nodes;
 * beyond the last entry: leaf 64, p 8). */
typedef struct {
    long long max_nodes;
    int leaf_cap;
    int order_p;
} afmpb_tuning_entry;

typedef struct {
    int status;                   /* AFMPB_OK, AFMPB_E_PENDING, or the error     */
    long long n_nodes;
    double energy;                /* polar energy, kcal/mol                      */
    afmpb_solve_info info;        /* ms_total = submit -> completion             */
    long long device_bytes;       /* device memory the request held              */
    double ms_admit;              /* submit -> admitted (setup starts)           */
    double ms_ready;              /* submit -> set up (first GMRES chunk issued) */
    double ms_done;               /* submit -> finished                          */
    char message[128];            /* error text ("" on success)                  */
} afmpb_result;

typedef struct {
    long long queued, active, completed, failed;
    long long device_bytes, device_bytes_peak;
} afmpb_server_counts;

/* Starts a server on `device` with setup_threads threads that build admitted
 * requests and one stepping thread.  setup_threads must be 1: parallel setup
 * is switched off until a host crash seen with several setup threads is
 * understood (AFMPB_E_INVALID otherwise).  params as for
 * afmpb_set_molecule, except that order_p == 0 / leaf_cap == 0 select per
 * request from the tuning table.  hip_stream (may be NULL): a stream of the
 * caller; the device work of each request starts only after the work that
 * was queued on it when the request was submitted.  Each request runs on a
 * stream of its own.  Errors: AFMPB_E_INVALID. */
afmpb_status afmpb_server_create(const afmpb_params *params,
                                 long long hbm_budget_bytes, int max_active,
                                 int setup_threads, int device, void *hip_stream,
                                 afmpb_server **out);

/* Replaces the tuning table (n entries, copied). */
afmpb_status afmpb_server_set_tuning(afmpb_server *s, int n,
                                     const afmpb_tuning_entry *table);

/* Queues a request (inputs copied) and returns its ticket.  Mesh errors are
 * reported on the request's result. */
afmpb_status afmpb_server_submit(afmpb_server *s, const afmpb_molecule *m,
                                 unsigned long long *ticket);

/* Result of a request.  wait != 0 blocks until it has finished.  Returns
 * AFMPB_E_PENDING (and fills status/timings so far) while it runs; once
 * finished returns AFMPB_OK, fills *out (out->status holds the request's own
 * outcome) and copies f, h [n_nodes] (physical units, caller order; either
 * may be NULL), and releases the ticket.  Unknown ticket: AFMPB_E_INVALID. */
afmpb_status afmpb_server_poll(afmpb_server *s, unsigned long long ticket,
                               int wait, afmpb_result *out, double *f,
                               double *h);

/* Cancels a request: a queued one finishes at once, a running one at its
 * next GMRES chunk, with status AFMPB_E_CANCELLED. */
afmpb_status afmpb_server_cancel(afmpb_server *s, unsigned long long ticket);

afmpb_status afmpb_server_stats(afmpb_server *s, afmpb_server_counts *out);

/* Stops the threads, cancels queued requests and frees everything.  Results
 * not yet polled are discarded.  NULL is accepted. */
afmpb_status afmpb_server_destroy(afmpb_server *s);

#ifdef __cplusplus
}
#endif
#endif /* AFMPB_H */

/*
 * topomg — multigrid-preconditioned conjugate gradients for SIMP-penalised
 * linear elasticity on uniform quad (Q4) / hex (Hex8) grids, on one AMD
 * Instinct MI355X (gfx950).
 *
 * The library solves K(rho) u = f, the finite-element equilibrium equation of
 * the compliance problem (Sec. 2 of Peetz & Elbanna, "On the use of Multigrid
 * Preconditioners for Topology Optimization"), with
 *   K(rho)  = sum_e E(rho_e) L_e^T KE L_e,
 *   E(rho)  = Emin + (E0 - Emin) rho^p              (modified SIMP, Sec. 2),
 * by conjugate gradients (Sec. 3.1) preconditioned with one multigrid V-cycle
 * (Algorithm 1) whose hierarchy uses shape-function prolongation and Galerkin
 * coarse operators A^{i+1} = P^T A^i P on the finest levels (Sec. 3.2) and,
 * optionally, smoothed aggregation on the coarser ones (the hybrid of
 * Sec. 4.3 / 4.4).  The V-cycle may run in FP32 inside an FP64 flexible CG.
 *
 * Conventions shared by every entry point
 *   mesh     nel[0..dim-1] elements per axis, square/cubic elements of edge h.
 *            node (i,j[,k]) = i + (nx+1)(j + (ny+1)k);  dof = dim*node + c;
 *            element (ex,ey[,ez]) = ex + nx(ey + ny ez).
 *            Element local node order: 2D counter-clockwise from the lower-left
 *            corner; 3D bottom face (z = ez) counter-clockwise, then top face.
 *   2D       plane stress, unit thickness.
 *   supports homogeneous Dirichlet conditions on a list of dof ids.  The
 *            operator solved is K~ = M K M + (I - M) (M = mask of free dofs),
 *            so u = 0 on supported dofs and loads given there are ignored.
 *   memory   "_dev" pointers are device memory, everything else host memory.
 *            The caller owns every buffer it passes; the library keeps no
 *            caller pointer past the call that received it.  A hierarchy owns
 *            the device memory it allocates until tm_destroy: from the
 *            tm_allocator given to tm_setup, else from hipMalloc.
 *   streams  `stream` is a hipStream_t (NULL = default stream).  All device
 *            work of a call is ordered on that stream.  Calls that return
 *            host-visible results synchronise that stream before returning.
 *   errors   Negative status: the call failed and outputs are undefined;
 *            tm_last_error() gives a message (per thread).  Positive status:
 *            a warning, outputs are valid.  Arguments are validated before any
 *            device work starts.
 *   threads  Distinct hierarchies may be used from distinct threads.  One
 *            hierarchy may run several solves at once only through distinct
 *            solve states (tm_solve_begin) on distinct streams.
 */
#ifndef TOPOMG_H
#define TOPOMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TM_OK = 0,
    TM_NOT_CONVERGED = 1,      /* iteration limit reached; u is the last iterate   */
    TM_ERR_ARG = -1,           /* invalid argument                                 */
    TM_ERR_OOM = -2,           /* device allocation failed                         */
    TM_ERR_DEVICE = -3,        /* HIP runtime error                                */
    TM_ERR_NOT_SPD = -4,       /* coarsest operator is not positive definite       */
    TM_ERR_BREAKDOWN = -5,     /* CG breakdown: p^T K p <= 0 or z^T r <= 0         */
    TM_ERR_STATE = -6          /* call out of order (e.g. a state already ended)   */
} tm_status;

typedef struct { int32_t dim; int32_t nel[3]; double h; } tm_mesh;
typedef struct { double p, E0, Emin, nu; } tm_material;
typedef struct { int64_t n; const int64_t* dofs; } tm_bcs;      /* host array of n dof ids */

enum { TM_SMOOTH_BLOCK_JACOBI = 0,   /* point-block (one block per node), Sec. 4.1 */
       TM_SMOOTH_POINT_JACOBI = 1,   /* diag(A) as printed in Algorithm 1           */
       TM_SMOOTH_CHEBYSHEV = 2 };    /* Jacobi-preconditioned Chebyshev, Sec. 4.1   */
enum { TM_OUTER_FCG = 0,             /* flexible CG, beta = -z^T q / p^T q          */
       TM_OUTER_PCG = 1 };           /* standard PCG, beta = z_k^T r_k / z_{k-1}^T r_{k-1} */
enum { TM_LEVEL_FINE = 0, TM_LEVEL_GEOMETRIC = 1, TM_LEVEL_AGGREGATION = 2 };

typedef struct {
    int32_t n_levels;      /* levels including the fine grid; 0 = automatic                      */
    int32_t n_geometric;   /* geometric levels including the fine grid; 0 = all geometric;
                              otherwise smoothed aggregation continues below level n_geometric-1 */
    int32_t max_coarse;    /* automatic depth: stop at the first level with fewer dofs (1000)    */
    int32_t smoother;      /* TM_SMOOTH_*                                                        */
    int32_t nu_pre;        /* pre-smoothing sweeps (>= 1)                                        */
    int32_t nu_post;       /* post-smoothing sweeps (>= 1)                                       */
    double  omega;         /* Jacobi weight (0.5)                                                */
    double  sa_beta;       /* strength threshold beta (0.003)                                    */
    int32_t vcycle_fp;     /* 32: FP32 V-cycle (FP64 outer loop); 64: FP64 everywhere            */
    int32_t outer;         /* TM_OUTER_FCG or TM_OUTER_PCG                                        */
    int32_t max_iters;     /* outer iteration limit (1000)                                        */
    int32_t check_every;   /* host convergence check period in iterations; 0 = adaptive          */
    int32_t fine_mfma;     /* 1: FP32 3D fine operator contracts KE on the matrix cores
                              (v_mfma_f32_4x4x1, KE broadcast from 12 registers, two nodes
                              stacked in z per lane); 0 (default): vector FMAs with KE
                              symmetry-class values in scalar registers.  Same operator either
                              way; only the rounding order differs                           */
    double  cheb_lower;    /* Chebyshev smoothing interval [cheb_lower, 1.1] x lambda, lambda =
                              power estimate of the largest eigenvalue of D^-1 A (0.1)        */
    int32_t adapt_iters;   /* automated hybrid (Sec. 4.4): when a solve takes more than this
                              many iterations, the next tm_update_density turns the coarsest
                              geometric level into smoothed-aggregation levels (down to 2
                              geometric levels, max_coarse as usual).  0 (default): off      */
    int32_t cheb_warm_steps; /* Chebyshev smoothing: a tm_update_density starts each geometric
                              level's power estimate from that level's last estimate vector and
                              runs this many steps (1..12) instead of 12 from the fixed start;
                              aggregation levels and the first setup always start cold.
                              0 (default): every setup runs 12 steps from the fixed start     */
    int32_t stencil_kernel; /* operator kernel of the geometric coarse levels: 0 (default) by
                              level size (levels of at least 256 workgroups of nodes take the
                              large-level kernel, smaller ones the latency-bound form); 1: the
                              large-level kernel on every level; 2: the small-level form on
                              every level; 3: as 0, but level 1 of a 3D grid with even element
                              counts in the FP32 V-cycle applied from the fine moduli (the
                              Galerkin product element by element in the tensor-product form,
                              no stored stencil read; slower than the stored stencil on the
                              grids measured).  Same operator either way                    */
    int32_t sa_lds;         /* aggregation setup: 0 (default) keeps a Galerkin product row's sums,
                              an aggregate's Gram-Schmidt rows and a prolongator row's blocks in
                              LDS when they fit; 1: never (block by block, in device memory).
                              The levels are bitwise the same either way                     */
    int32_t fine_tensor;    /* form of the 3D fine operators (FP32 in the V-cycle, FP64 for the
                              outer q = K~p and the FP64 V-cycle): 1 (default) the tensor-product
                              form: in per-axis sum / difference modes of an element's corner
                              values KE has 45 couplings instead of 576 entries; a workgroup
                              marches 32 x 8 element columns up a range of node planes and adds
                              each node's corner values through LDS; n >= 2: the same with n
                              node planes per workgroup (default: from the grid's size); 0: the
                              node gather (27 neighbours, KE class values).  fine_mfma = 1 takes
                              precedence for the FP32 operator.  Same operator; only the
                              rounding differs                                                */
} tm_options;

/* Source of a hierarchy's device memory (levels, solve states, work vectors,
 * aggregation levels, eigensolver workspace), e.g. a framework's caching
 * allocator.
 *   alloc(bytes, stream, ctx) returns `bytes` of device memory on the current
 *     device, aligned to 256 bytes, for use on `stream` (the stream of the call
 *     that needs it), or NULL (the call then fails with TM_ERR_OOM);
 *   free(ptr, stream, ctx) takes back a block from alloc.  The library calls it
 *     only after synchronising the device, so no queued work uses the block.
 *   ctx is passed through and must stay valid until tm_destroy.
 * The callbacks are called from the thread that calls into the library, during
 * tm_setup, tm_update_density (aggregation levels), the first solve of a new
 * right-hand-side count, tm_vcycle, tm_stress_stiffness, tm_eigs and
 * tm_destroy. */
typedef struct {
    void* (*alloc)(size_t bytes, void* stream, void* ctx);
    void (*free)(void* ptr, void* stream, void* ctx);
    void* ctx;
} tm_allocator;

typedef struct tm_hierarchy tm_hierarchy;       /* opaque */
typedef struct tm_solve_state tm_solve_state;   /* opaque */

/* Fill `o` with the defaults listed above (FCG, FP32 V-cycle, block Jacobi 1/1, omega 0.5). */
void tm_default_options(tm_options* o);

/* Device bytes a hierarchy plus workspace for n_rhs concurrent right-hand sides
 * will hold, computed on the host only (admission control). */
tm_status tm_plan_bytes(const tm_mesh* mesh, const tm_options* opts, int32_t n_rhs, size_t* bytes);

/* Build the multigrid hierarchy for densities rho_dev[n_el] (FP64, in [0,1]):
 * SIMP moduli, fine point-block diagonal, geometric Galerkin levels, optional
 * smoothed-aggregation levels, coarsest Cholesky factor (Secs. 2, 3.2, 4).
 * Each geometric coarsening takes an axis of n elements to ceil(n/2) (Sec. 4.3);
 * for odd n the last coarse element is a single fine element (aggregation
 * levels below such a chain take the rigid-body modes at the true node positions).
 * Errors: TM_ERR_ARG (bad mesh/material/options, an axis that would be coarsened
 * below one element, dof id out of range), TM_ERR_NOT_SPD, TM_ERR_OOM.
 * rho values are checked on the device (finite and in [0,1]).
 * alloc: the hierarchy's device memory source for its whole life (NULL:
 * hipMalloc / hipFree); TM_ERR_ARG if it is given without both callbacks. */
tm_status tm_setup(const tm_mesh* mesh, const tm_material* mat, const double* rho_dev,
                   const tm_bcs* bcs, const tm_options* opts, const tm_allocator* alloc, void* stream,
                   tm_hierarchy** out);

/* Numeric re-setup for new densities on the same mesh, supports and options
 * (a design iteration): the structure and all allocations are reused.  For a
 * hierarchy without aggregation levels the call only enqueues work on `stream`
 * and returns; what the device finds (densities outside [0,1], a block or the
 * coarsest operator not SPD) is then reported by the next solve on this
 * hierarchy (TM_ERR_ARG / TM_ERR_NOT_SPD), which must be ordered after it.
 * With aggregation levels (whose sizes depend on the values) it waits and
 * reports those errors itself. */
tm_status tm_update_density(tm_hierarchy* h, const double* rho_dev, void* stream);

/* Solve K~ u_k = M f_k for k < n_rhs.  f_dev and u_dev hold n_rhs vectors of
 * n_dof FP64 values, one after the other.  If use_u0, u_dev holds the start
 * vectors (warm start, Sec. 4); otherwise the start is zero.  Stops when the
 * recursive residual satisfies ||r|| <= rtol ||M f||.  Host outputs per
 * right-hand side: iterations, compliance f^T u (Sec. 2), and the true
 * relative residual ||M f - K~ u|| / ||M f||.  Any output pointer may be NULL.
 * Returns TM_NOT_CONVERGED if some right-hand side hit max_iters (u is then
 * the last iterate); TM_ERR_ARG if a load or start vector holds an infinity or
 * a NaN (found on the device at the first step); TM_ERR_BREAKDOWN if p^T K~ p
 * <= 0 or, for PCG, z^T r <= 0 (a V-cycle that is not positive definite, e.g.
 * an over-relaxed smoother).  tm_last_error() names the right-hand side.
 * The right-hand sides share every launch (several load cases, Sec. 2 and
 * Sec. 4.2); each one's result is bitwise that of its own solve. */
tm_status tm_solve(tm_hierarchy* h, int32_t n_rhs, const double* f_dev, double rtol,
                   int32_t use_u0, double* u_dev, int32_t* iters, double* compliance,
                   double* relres, void* stream);

/* Design sensitivity of the summed compliances (Sec. 2; compliance is
 * self-adjoint, so no second solve is needed):
 *   dc_e = -p rho_e^(p-1) (E0 - Emin) sum_k u_k,e^T KE u_k,e
 * for the densities of the current design (tm_setup / tm_update_density).
 * u_dev holds n_rhs solutions of n_dof FP64 values one after the other (as
 * returned by tm_solve); dc_dev receives n_el FP64 values in element order.
 * Both are device buffers owned by the caller.  Enqueued on `stream`; the call
 * does not wait for it.  TM_ERR_ARG for a NULL handle or buffer or n_rhs < 1. */
tm_status tm_compliance_sensitivity(tm_hierarchy* h, int32_t n_rhs, const double* u_dev, double* dc_dev,
                                    void* stream);

/* Linear density filter (Sec. 2: filtered densities rho = S alpha; Sec. 4: radius
 * 1.5 element sizes).  S[e][i] = H[e][i] / sum_j H[e][j] over the elements i of the
 * grid, H[e][i] = max(0, radius - |c_e - c_i|), c = element centres in units of
 * the element size.
 *   transpose = 0: out = S in    (design variables -> filtered densities)
 *   transpose = 1: out = S^T in  (sensitivities w.r.t. rho -> w.r.t. alpha)
 * in_dev, out_dev: n_el FP64 device buffers in element order (x fastest), owned by
 * the caller; they must not overlap.  radius in (0, 4].  Enqueued on `stream`; the
 * call does not wait.  TM_ERR_ARG for a bad mesh, radius or NULL buffer. */
tm_status tm_density_filter(const tm_mesh* mesh, double radius, int32_t transpose, const double* in_dev,
                            double* out_dev, void* stream);

/* tm_density_filter for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same filter, same arguments and same results, but the transpose keeps its
 * intermediate W^-1 in (one FP64 value per element) in a fixed device array of
 * the library instead of stream-ordered scratch.  The call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine).
 *   Limit: at most 8,388,608 elements (the array is 64 MiB; each GPU the library
 *   runs on holds its own copy until the process ends); larger meshes get
 *   TM_ERR_ARG before any device work.
 *   Sharing: every call on one GPU uses that GPU's array, so calls whose device
 *   work overlaps on one GPU (different streams, or different threads, without
 *   ordering) race and give wrong results; order them on one stream.  Every
 *   entry the transpose reads is written earlier in the same call, so no state
 *   carries over between calls.
 *   The first call on a device looks up the array's address on that device
 *   (the device must be current).  Errors as tm_density_filter. */
tm_status tm_density_filter_noalloc(const tm_mesh* mesh, double radius, int32_t transpose, const double* in_dev,
                                    double* out_dev, void* stream);

/* ---- stability eigenproblem (Sec. 2 stability maximisation; Sec. 3 eigensolvers,
 * Algorithm 2 generalized Davidson; Sec. 4 column example) ------------------ */

/* Stress-stiffness matrix of the displacements u_dev (n_dof FP64, device, e.g. a
 * tm_solve result) for the densities of the current design:
 *   K_sigma = -sum_e E_sigma(rho_e) L_e^T (g_e (x) I_dim) L_e,
 *   E_sigma(rho) = E0 rho^p for rho >= rho_min (0.1 in Sec. 2), 0 below,
 *   g_e[a][b] = sum over the 2^dim Gauss points of w |J| grad N_a^T sigma grad N_b,
 * sigma the unit-modulus stress of u_e (plane stress in 2D).  The paper does not
 * write K_sigma out: this is the textbook geometric stiffness, with the sign
 * that gives compressive states positive eigenvalues of K_sigma Phi = lambda K Phi
 * (lambda = 1 / critical load factor).  Supported rows and columns are removed
 * (K_sigma~ = M K_sigma M).  The hierarchy keeps the matrix (a scalar nodal
 * stencil, 3^dim FP64 per node) until the next call; tm_update_density makes it
 * stale.  Enqueued on `stream`, which must be ordered after the work that wrote
 * u_dev; the call does not wait.  TM_ERR_ARG for a NULL handle or buffer or
 * rho_min outside [0, 1]; TM_ERR_OOM. */
tm_status tm_stress_stiffness(tm_hierarchy* h, const double* u_dev, double rho_min, void* stream);

/* y = K_sigma~ x (device FP64 vectors of n_dof, not overlapping), with the matrix of
 * the last tm_stress_stiffness.  Waits for completion.  TM_ERR_STATE if there is
 * no current stress-stiffness matrix. */
tm_status tm_apply_stress_stiffness(tm_hierarchy* h, const double* x_dev, double* y_dev, void* stream);

typedef struct tm_eig_options {
    int32_t nev;        /* eigenpairs wanted, the largest eigenvalues (6 in Sec. 4)          */
    int32_t j_min;      /* search-space size kept at a restart (10 in Sec. 3); nev < j_min   */
    int32_t j_max;      /* search-space size that triggers a restart (25); j_min < j_max <= 32 */
    int32_t max_iters;  /* search-space expansions (preconditioner calls) at most            */
    double tol;         /* a pair converges when ||K_s q - theta K q|| / (|theta| ||K q||)
                           falls below tol (1e-6, Sec. 4) ...                                */
    double stag_tol;    /* ... or when theta changes by less than stag_tol |theta| between
                           consecutive iterations (1e-13, Sec. 4)                           */
    int32_t precond_fp; /* 32: FP32 V-cycle as the preconditioner M, 64: FP64 V-cycle       */
} tm_eig_options;

/* Fill `o` with nev 6, j_min 10, j_max 25, max_iters 1000, tol 1e-6, stag_tol
 * 1e-13, precond_fp 32. */
void tm_default_eig_options(tm_eig_options* o);

/* The nev largest eigenvalues of K_sigma~ Phi = lambda K~ Phi by generalized
 * Davidson (Algorithm 2) with one V-cycle of the hierarchy as the preconditioner,
 * using the matrix of the last tm_stress_stiffness.
 *   v0_dev   n_init start vectors (1 <= n_init <= j_max), n_dof FP64 each, one after
 *            the other (device); entries on supported dofs are ignored.  Previous
 *            eigenvectors make good start vectors (Sec. 4).
 *   lambda   host, nev values, descending.
 *   phi_dev  device, nev eigenvectors of n_dof one after the other, normalised
 *            Phi^T K~ Phi = I (may be NULL).
 *   iters    host, expansions done (may be NULL); n_conv: converged pairs (may be NULL).
 * Method as implemented: Gram-Schmidt in the K~ inner product (classical, repeated
 * once when the norm drops below 1/sqrt(2) of its value), the Ritz pairs of
 * V^T K_sigma~ V, pairs converge in descending order and stay in the space, a
 * restart keeps the j_min leading Ritz vectors.  Waits for completion.  The
 * hierarchy keeps the search space (n_dof x j_max FP64) for later calls.
 * Returns TM_NOT_CONVERGED if fewer than nev pairs converged within max_iters;
 * TM_ERR_STATE without a current stress-stiffness matrix; TM_ERR_ARG for bad
 * options, start vectors that are dependent in the K~ inner product, or NULL
 * pointers; TM_ERR_BREAKDOWN if a correction lies in the search space. */
tm_status tm_eigs(tm_hierarchy* h, const tm_eig_options* o, int32_t n_init, const double* v0_dev,
                  double* lambda, double* phi_dev, int32_t* iters, int32_t* n_conv, void* stream);

/* Iteration-level control for a scheduler (continuous batching).
 * begin:   copies f, sets up the start vector on `stream` and returns a state
 *          bound to (h, stream, u_dev); u_dev must stay valid until end.
 * advance: enqueues up to k further iterations on the state's stream without
 *          waiting.
 * poll:    non-blocking; *done = 1 once every right-hand side has stopped, 0 when
 *          the enqueued iterations have finished without that, -1 while they
 *          are still running.
 * batch_iterate: k further iterations of n states (of one or several
 *          hierarchies), enqueued on `stream` as grouped launches: the
 *          right-hand sides of all states whose hierarchies have the same level
 *          structure and options (level kinds and sizes, smoother, sweeps,
 *          precision, outer method, element stiffness) advance together, each
 *          operation of an iteration (operators and transfers per level,
 *          coarsest solve, Krylov updates and reductions) one launch for up to
 *          8 right-hand sides; aggregation levels, whose operators differ per
 *          hierarchy, are applied per right-hand side in the same sequence.
 *          `stream` first waits for the work queued on each state's own stream,
 *          and each state's stream waits for the batch, so later calls on a
 *          state stay ordered.  Every right-hand side computes exactly what it
 *          computes alone.  A state may appear only once in the list.
 * end:     waits, writes the outputs of tm_solve and releases the state (its
 *          device buffers stay with the hierarchy for the next begin).  Each
 *          begin, advance and batch_iterate also computes the outputs (true
 *          residual, compliance) of the right-hand sides that stopped in it, as
 *          the same kernels as end's; after a poll that reported done = 1, end
 *          therefore launches and waits for nothing.
 * The right-hand sides of one state always share launches (also in tm_solve). */
tm_status tm_solve_begin(tm_hierarchy* h, int32_t n_rhs, const double* f_dev, double rtol,
                         int32_t use_u0, double* u_dev, void* stream, tm_solve_state** st);
tm_status tm_solve_advance(tm_solve_state* st, int32_t k_iters);
tm_status tm_solve_poll(tm_solve_state* st, int32_t* done);
tm_status tm_batch_iterate(int32_t n, tm_solve_state* const* st, int32_t k_iters, void* stream);
tm_status tm_solve_end(tm_solve_state* st, int32_t* iters, double* compliance, double* relres);

/* ---- parity and inspection (tests) --------------------------------------- */
/* y = A_level x on the device, FP64 (fp = 64) or FP32 (fp = 32) data.  Level 0
 * is K~ (matrix-free), level l > 0 the stored coarse operator. */
tm_status tm_apply(tm_hierarchy* h, int32_t level, int32_t fp, const void* x_dev, void* y_dev,
                   void* stream);
/* x = V(M b): one V-cycle of Algorithm 1 from x = 0 on level 0, in the given precision
 * (as applied inside tm_solve: entries of b on supported dofs are ignored, and x
 * is zero there). */
tm_status tm_vcycle(tm_hierarchy* h, int32_t fp, const void* b_dev, void* x_dev, void* stream);
/* Level shape: rows (dofs), stored nonzeros in CSR form, TM_LEVEL_*, dofs per node. */
tm_status tm_level_info(const tm_hierarchy* h, int32_t level, int64_t* n_rows, int64_t* nnz,
                        int32_t* kind, int32_t* block);
int32_t tm_num_levels(const tm_hierarchy* h);
/* Level operator (level >= 1) as CSR, FP64 values, ascending columns (host buffers
 * of n_rows+1, nnz, nnz entries).  The fine level (matrix-free) is not exported. */
tm_status tm_export_csr(const tm_hierarchy* h, int32_t level, int64_t* rowptr, int32_t* colidx,
                        double* vals);
/* Prolongator from level+1 to level as CSR (rows: dofs of `level`).  Call with
 * NULL arrays to get *nnz first. */
tm_status tm_export_prolongator(const tm_hierarchy* h, int32_t level, int64_t* n_rows,
                                int64_t* nnz, int64_t* rowptr, int32_t* colidx, double* vals);
/* Aggregate id of every node of an aggregation input level (host int32[n_nodes]). */
tm_status tm_export_aggregates(const tm_hierarchy* h, int32_t level, int32_t* agg_of_node);
/* Point-block diagonal inverse of a level, FP64, [node][bs*bs] row-major blocks. */
tm_status tm_export_dinv(const tm_hierarchy* h, int32_t level, double* dinv);
/* The coarsest level's inverse as the V-cycle applies it (Sec. 3.2 coarsest
 * solve; formed at setup from the FP64 Cholesky factor as L^-T L^-1), n x n
 * FP64 row-major into a host buffer, n = rows of the last level.  Waits for the
 * device. */
tm_status tm_export_coarse_inverse(const tm_hierarchy* h, double* ainv);
/* Element-to-node table of a mesh (host int32[n_el * 2^dim], local order above). */
tm_status tm_export_connectivity(const tm_mesh* mesh, int32_t* conn);
/* Device bytes held by the hierarchy (not counting solve states). */
tm_status tm_hierarchy_bytes(const tm_hierarchy* h, size_t* bytes);

/* Kernel timing for roofline reporting: when enabled, every launch of a kernel
 * class inside solves of `h` is bracketed by HIP events on its own stream:
 * class 0 = the outer FP64 operator q = K~p, class 1 = the fine-level operator
 * of the V-cycle (residual / smoothing sweeps), class 2 = the operator of the
 * first coarse level.  read returns the launch count and the summed event time
 * in milliseconds, then resets.  Timing adds event records between launches;
 * it is meant for a separate, profiled solve. */
tm_status tm_kernel_timing(tm_hierarchy* h, int32_t kernel_class, int32_t enable);
tm_status tm_kernel_timing_read(tm_hierarchy* h, int32_t kernel_class, int64_t* launches,
                                double* total_ms);

void tm_destroy(tm_hierarchy* h);
const char* tm_status_string(tm_status s);
const char* tm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TOPOMG_H */

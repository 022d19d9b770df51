/*
 * cutbddc: BDDC-preconditioned conjugate gradients for unfitted (cut-cell)
 * Q1 finite elements on one AMD Instinct MI355X (gfx950).
 *
 * Method: S. Badia, F. Verdugo, "Robust and scalable domain decomposition
 * solvers for unfitted finite element methods" (arXiv:1703.06323).
 *   - Problem: find u in V-bar with A-bar u = b, A-bar = sum_e A_e (Sect. 2.2),
 *     strong Dirichlet data on the mesh-aligned boundary (Sect. 5.1).
 *   - Domain: Omega = {phi > 0}, phi(x) = min_i(|x - c_i| - r_i) on the unit
 *     cube (level-set geometry, Sect. 2.1); background mesh of N^3 cells.
 *   - Subdomains: aggregation of active cells in uniform s^3 blocks (Sect. 2.1).
 *   - Preconditioner: M = I0 A0^-1 I0^T + Q A~^-1 Q^T, Q = E W (eq. bddc),
 *     coarse DOFs = object means (eq. coarse-dofs), BDDC(cef) or BDDC(ce),
 *     topological (eq. weighting) or stiffness (eq. alge-weighting) weights,
 *     standard objects (Sect. 3.2), variant 1 (cut coarse edges split,
 *     Sect. 4.4) or variant 2 (coarse edges split where the stiffness
 *     weighting coefficient changes, Sect. 4.5).
 *   - Solver: PCG with |r|_2 < rtol |b|_2 (Sect. 5.1).
 *
 * Conventions for every entry point:
 *   - Return value: CB_OK (0) on success, a negative CB_ERR_* code on
 *     failure; cb_last_error() then gives a message (thread-local).  No
 *     exception crosses this interface and no entry point exits the process.
 *   - Pointers named *_dev are device pointers (HBM) owned by the caller; the
 *     library never frees or keeps them after the call returns.  Host inputs
 *     are copied before the call returns.
 *   - All device work runs on the HIP stream given to cb_setup; calls that
 *     return host values synchronise that stream.
 *   - Grid layouts: cells are numbered i + N (j + N k), grid nodes
 *     I + (N+1)(J + (N+1) K) with x fastest.  DOF vectors hold the active
 *     interior nodes in ascending node order (cb_info.n_dof entries).
 *   - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef CUTBDDC_H
#define CUTBDDC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum cb_status {
  CB_OK = 0,
  CB_ERR_ARG = -1,             /* invalid argument (sizes, options, NaN/<=0 kappa)     */
  CB_ERR_SINGULAR = -2,        /* an active component touches no Dirichlet node        */
  CB_ERR_NOT_SPD = -3,         /* a local or coarse Cholesky met a non-positive pivot  */
  CB_ERR_NO_CONVERGENCE = -4,  /* max_iter reached; best iterate returned              */
  CB_ERR_DEVICE = -5,          /* a HIP runtime call failed                            */
  CB_ERR_STATE = -6,           /* call out of order (e.g. solve before factor)         */
  CB_ERR_OOM = -7              /* device allocation failed                             */
};

enum cb_weighting { CB_W_CARDINALITY = 0, CB_W_STIFFNESS = 1 };
enum cb_objects { CB_OBJ_CEF = 0, CB_OBJ_CE = 1 };
enum cb_variant { CB_CV_STANDARD = 0, CB_CV_V1 = 1, CB_CV_V2 = 2 };
enum cb_precision { CB_FP64 = 0, CB_FP32_LOCAL = 1 };

typedef struct {
  int32_t n_cells;             /* N: background cells per axis on [0,1]^3, h = 1/N       */
  int32_t sub_cells;           /* s: subdomain block size in cells; must divide N        */
  int32_t n_balls;             /* number of balls removed from the cube (may be 0)       */
  const double* ball_centres;  /* host, [n_balls * 3] (x, y, z per ball)                  */
  const double* ball_radii;    /* host, [n_balls], > 0                                    */
  const double* kappa;         /* host, [N^3] per-cell conductivity > 0, or NULL (= 1)    */
  int32_t weighting;           /* cb_weighting                                            */
  int32_t objects;             /* cb_objects                                              */
  int32_t coarse_variant;      /* cb_variant                                              */
  int32_t local_precision;     /* cb_precision: subdomain factor/solves in FP64 or FP32   */
  int32_t full_elements;       /* test flag: integrate every active cell as uncut         */
  int32_t cut_boundary;        /* ball surfaces: 0 homogeneous Neumann; 1 homogeneous     */
                               /* Dirichlet imposed by Nitsche's method with beta_e =     */
                               /* 2 lambda_max (Sect. 2.2, eq. local-eigenvals)           */
} cb_problem;

typedef struct {
  int64_t n_dof;               /* active interior nodes (unknowns)                        */
  int64_t n_active;            /* active cells                                            */
  int64_t n_cut;               /* cut cells                                               */
  int64_t n_cut_stored;        /* cut cells with stored matrices (0 with full_elements)   */
  int32_t n_sub;               /* subdomains (m^3, empty blocks included)                 */
  int32_t n_coarse;            /* coarse DOFs                                             */
  int32_t n_objects;           /* interface objects (selected or not)                     */
  int32_t n_iface;             /* interface DOFs                                          */
  int32_t max_local_dofs;      /* largest n_omega                                         */
  int32_t max_coarse_per_sub;  /* largest number of coarse DOFs touching one subdomain    */
  int32_t n_fp64_fallbacks;    /* FP32-local subdomains refactored in FP64                */
  int32_t factored;            /* 1 once cb_factor succeeded                              */
  int64_t sum_nI2;             /* sum over subdomains of n_I^2 (Dirichlet inverse size)   */
  int64_t sum_nG2;             /* sum over subdomains of n_G^2 (interface operator size)  */
  int64_t sum_nI;              /* sum of interior DOF counts                              */
  int64_t sum_nG;              /* sum of interface DOF counts (with multiplicity)         */
  double flops_local_chol;     /* sum over subdomains of (n_I+n_G)^3/3 + n_I^3/3           */
  double t_integrate_ms;       /* last phase times (HIP events + host clock)              */
  double t_topology_ms;
  double t_factor_ms;
  double t_solve_ms;
  int64_t sum_nGnC;            /* sum over subdomains of n_G * (coarse DOFs touching it)  */
  int64_t n_nodes;             /* grid nodes (N+1)^3, summed over problems                */
  double lanczos_lmin;         /* extreme eigenvalue estimates of M A-bar from the last   */
  double lanczos_lmax;         /* solve's PCG coefficients (cb_pcg_history); 0 before one,
                                  and in cb_query of a batch context                      */
  int32_t coarse_separator;    /* cb_query after cb_factor: separator size when the coarse */
  int32_t coarse_octant_max;   /* problem is solved by nested dissection (one problem,     */
                               /* m >= 4 and n_coarse >= 1024, or CUTBDDC_COARSE=nd; the  */
                               /* largest octant block in the second field); 0 and 0 when */
                               /* it is a dense Cholesky of the whole coarse matrix        */
} cb_info;

typedef struct cb_ctx cb_ctx;

/* Classify cells and integrate cut cells (Sect. 2.1-2.2), number DOFs,
 * build subdomains, objects and coarse DOFs (Sect. 3.1-3.2, 4.4).
 * `stream` is a hipStream_t (NULL = default stream).  On success *out owns
 * all device buffers of the problem; release it with cb_destroy.
 * Errors: CB_ERR_ARG (N < 1, s does not divide N, bad option, radius <= 0,
 * kappa <= 0 or not finite), CB_ERR_SINGULAR (floating active component),
 * CB_ERR_DEVICE / CB_ERR_OOM. */
int cb_setup(const cb_problem* p, void* stream, cb_ctx** out);

/* Sub-assemble the local Neumann matrices (Sect. 3.1), compute weights
 * (eq. weighting / eq. alge-weighting), factor the local Dirichlet and
 * constrained Neumann problems, the coarse basis and the coarse matrix
 * (Sect. 3.3-3.4).  Errors: CB_ERR_STATE, CB_ERR_NOT_SPD, CB_ERR_DEVICE. */
int cb_factor(cb_ctx* c);

/* b = M_cut f (Q1 source with nodal values f on all (N+1)^3 grid nodes,
 * f_nodes_dev == NULL means f = 1), then PCG with M from x0 = 0 until
 * |r|_2 < rtol |b|_2 (Sect. 5.1).  u_dev: [n_dof] device output.
 * *iters = operator applies, *final_relres = |r|/|b| of the recursive
 * residual.  CB_ERR_NO_CONVERGENCE leaves the last iterate in u_dev. */
int cb_solve(cb_ctx* c, const double* f_nodes_dev, double* u_dev, double rtol,
             int32_t max_iter, int32_t* iters, double* final_relres);

/* Same PCG for an explicit right-hand side b_dev: [n_dof] (adjoint solves). */
int cb_solve_rhs(cb_ctx* c, const double* b_dev, double* u_dev, double rtol,
                 int32_t max_iter, int32_t* iters, double* final_relres);

/* Adjoint contraction for J(u) with dJ/du = A-bar lambda and kappa = exp(theta):
 * dJ_dtheta_dev[e] = -kappa_e lambda_e^T K_e u_e (per cell, 0 if inactive),
 * dJ_df_dev = M_cut^T lambda over all grid nodes.  Inputs [n_dof]. */
int cb_grad(cb_ctx* c, const double* u_dev, const double* lam_dev,
            double* dJ_dtheta_dev, double* dJ_df_dev);

/* Building blocks exposed for parity testing.  All vectors [n_dof], device. */
int cb_apply_operator(cb_ctx* c, const double* x_dev, double* y_dev);       /* y = A-bar x  */
int cb_apply_preconditioner(cb_ctx* c, const double* r_dev, double* z_dev); /* z = M r      */
int cb_load(cb_ctx* c, const double* f_nodes_dev, double* b_dev);           /* b = M_cut f  */

/* Manufactured-solution accuracy (Sect. 5.1): the exact solution
 * u = sin(k |x - x0|) (the paper takes k = 5 pi, x0 = the origin), with
 * strong Dirichlet data u on the cube faces and, on the ball surfaces,
 * Neumann data grad u . n (cut_boundary 0) or Dirichlet data u by Nitsche's
 * method (cut_boundary 1).  Single-problem contexts whose kappa is 1.
 * x0: host double[3].  Volume integrals use the kept points of the volume
 * rule, surface integrals the sphere rule of the Nitsche terms.
 * cb_manufactured_load: b_dev [n_dof] (device) = the load of f = -Lap u
 *   plus the surface data, minus A-bar applied to the Dirichlet lift; solve
 *   with cb_solve_rhs.
 * cb_manufactured_errors: *l2, *h1 (host) = the L2 and H1-seminorm errors
 *   of u_h = u_dev [n_dof] (device) plus the lift, over the kept points.
 * Errors: CB_ERR_ARG (null pointer, non-finite x0 or k, a given kappa),
 * CB_ERR_STATE (a batch context), CB_ERR_DEVICE / CB_ERR_OOM.  Both calls
 * allocate work buffers and synchronise the stream. */
int cb_manufactured_load(cb_ctx* c, const double* x0, double k, double* b_dev);
int cb_manufactured_errors(cb_ctx* c, const double* x0, double k, const double* u_dev,
                           double* l2, double* h1);

/* Totals over every problem of the context (one problem for cb_setup). */
int cb_query(const cb_ctx* c, cb_info* out);

/* ---- batches of independent problems -------------------------------------
 * Many independent meshes (the per-mesh problem statement of Sect. 2.2 for
 * each) held by one context, so that every kernel launch of setup, factor
 * and solve covers all of them: subdomains of all problems form one batch
 * of local factorisations, the coarse matrices are factored in groups of
 * equal padded order, and the PCG runs all problems in lock step with a
 * per-problem convergence flag on the device (a converged problem stops
 * changing; the iteration is replayed from a captured HIP graph).
 *
 * cb_setup_batch: problems[0..n) as in cb_setup; they must share sub_cells
 * and every option field (weighting, objects, coarse_variant,
 * local_precision, full_elements); N, balls and kappa are per problem.
 * Errors as cb_setup (the message names the problem), CB_ERR_ARG for n < 1
 * or differing options.  cb_factor factors all problems; cb_query returns
 * totals.  The single-problem entry points (cb_solve, cb_solve_rhs, cb_grad,
 * cb_apply_*, cb_load, cb_export_*) return CB_ERR_STATE on a context with
 * more than one problem. */
int cb_setup_batch(const cb_problem* problems, int32_t n, void* stream, cb_ctx** out);

/* Solves every problem k of the context: b_k = M_cut f_k, PCG with M until
 * |r_k| < rtol |b_k| (Sect. 5.1), each problem stopping on its own.
 * f_nodes_dev: host array of n device pointers to [(N_k+1)^3] nodal values
 * (the array or an entry may be NULL: f = 1).  u_dev: host array of n device
 * pointers to [n_dof_k] outputs.  iters, final_relres: host arrays [n] or
 * NULL.  Returns CB_ERR_NOT_SPD if some problem broke down, else
 * CB_ERR_NO_CONVERGENCE if some problem hit max_iter (every u_k still holds
 * its last iterate), else CB_OK.  Synchronises the context stream. */
int cb_solve_batch(cb_ctx* c, const double* const* f_nodes_dev, double* const* u_dev, double rtol,
                   int32_t max_iter, int32_t* iters, double* final_relres);

/* Counts of problem k of the context (fields as cb_info; times are 0). */
int cb_query_problem(const cb_ctx* c, int32_t k, cb_info* out);

/* Record of the last solve of problem k (0 for cb_setup contexts), kept on
 * the device by the convergence check of every PCG iteration (Sect. 5.1):
 * *n = iterations recorded (the first 1024 at most); alpha[j] and relres[j]
 * (|r_j| / |b| of the recursive residual) for j < n; beta[j] = rho_{j+1} /
 * rho_j, rho = r.z, for j < n - 1.  *lambda_min, *lambda_max = the extreme
 * eigenvalues of the Lanczos matrix of those n steps, estimates of the
 * spectrum of M A-bar (their quotient estimates its condition number; NaN
 * when the coefficients are not those of an SPD system).  Host outputs;
 * arrays hold cap entries, any output but n may be null.  Synchronises the
 * context stream.  Errors: CB_ERR_ARG, CB_ERR_STATE (no solve yet). */
int cb_pcg_history(const cb_ctx* c, int32_t k, int32_t cap, double* alpha, double* beta, double* relres,
                   int32_t* n, double* lambda_min, double* lambda_max);

/* The same estimates from given CG coefficients: n alphas (> 0) and n - 1
 * betas (>= 0), host arrays; the tridiagonal matrix has diagonal
 * 1/alpha_j + beta_{j-1}/alpha_{j-1} and off-diagonal sqrt(beta_j)/alpha_j,
 * and its extreme eigenvalues come from bisection on Sturm counts.  n = 0
 * gives (1, 1).  No GPU needed.  Errors: CB_ERR_ARG. */
int cb_lanczos_extremes(int32_t n, const double* alpha, const double* beta, double* lambda_min,
                        double* lambda_max);

/* Measurement hooks.  With profiling enabled the library brackets every
 * launch of the named kernel groups with HIP events on the context stream:
 * "apply_interior" (Dirichlet inverse products), "apply_neumann" (interface
 * operator products), "apply_A" (matrix-free operator), "coarse_gemv",
 * "local_cholesky" (the whole blocked Cholesky of the local matrices),
 * "local_inverse" (triangular inverses and products), "coarse_factor".
 * cb_profile_time synchronises the stream and returns the summed elapsed
 * time and the number of bracketed launches since profiling was enabled. */
int cb_profile(cb_ctx* c, int32_t enable);
int cb_profile_time(cb_ctx* c, const char* name, double* total_ms, int64_t* launches);
/* Per-launch durations (ms, in launch order) of the named group: at most
 * `cap` values are written to ms (host array); *n receives the number of
 * launches recorded.  Synchronises the stream. */
int cb_profile_launches(cb_ctx* c, const char* name, double* ms, int64_t cap, int64_t* n);
/* Average duration (ms) of one launch of a preconditioner kernel over `reps`
 * back-to-back launches on the context stream, bracketed by two HIP events
 * (so that launch gaps do not count): which = 0 the Dirichlet inverse
 * product (apply_interior, input r), 1 the interface operator product
 * (apply_neumann).  The kernels write only the context's scratch vectors.
 * Needs a factored context; synchronises the stream.  CB_ERR_STATE before
 * cb_factor, CB_ERR_ARG for reps < 1 or an unknown kernel. */
int cb_time_kernel(cb_ctx* c, int32_t which, int32_t reps, double* avg_ms);

/* Host copies of the integer data of the discretisation (bit-exact parity).
 * Each output pointer may be NULL; sizes come from cb_query / cb_export_sizes.
 *  cell_status [N^3]      0 inactive, 1 cut, 2 interior
 *  cell_count  [N^3]      kept points per cell
 *  dof_node    [n_dof]    grid node of each DOF
 *  card        [n_dof]    |S(xi)|: number of subdomains containing the DOF
 *  obj_ptr     [n_objects+1], obj_dofs [n_iface]: DOFs per object (ascending)
 *  obj_type    [n_objects] 0 corner, 1 edge, 2 face
 *  coarse_of_obj [n_objects] coarse id or -1 */
int cb_export_indexing(const cb_ctx* c, uint8_t* cell_status, int32_t* cell_count,
                       int64_t* dof_node, int32_t* card, int64_t* obj_ptr,
                       int64_t* obj_dofs, int8_t* obj_type, int32_t* coarse_of_obj);

/* The same arrays for problem k of a context (any number of problems; sizes
 * from cb_query_problem).  Numbering is local to the problem: cells, nodes
 * and DOFs of problem k start at 0.  CB_ERR_ARG for k out of range. */
int cb_export_problem_indexing(const cb_ctx* c, int32_t k, uint8_t* cell_status, int32_t* cell_count,
                               int64_t* dof_node, int32_t* card, int64_t* obj_ptr, int64_t* obj_dofs,
                               int8_t* obj_type, int32_t* coarse_of_obj);

/* Local DOFs of every subdomain of problem k (Sect. 3.1: the DOFs of the
 * nodes of the subdomain's active cells), host copies:
 *  sub_ptr  [n_sub+1]         CSR offsets, subdomains in id order
 *                             Bx + m (By + m Bz), empty blocks included
 *  sub_dofs [sub_ptr[n_sub]]  DOF ids, ascending within a subdomain
 * sub_dofs may be NULL (sizes only).  CB_ERR_ARG for k out of range. */
int cb_export_subdomains(const cb_ctx* c, int32_t k, int64_t* sub_ptr, int64_t* sub_dofs);

/* Cut-cell reference matrices (kappa = 1, h = 1), host copies, packed upper
 * triangles row by row (36 values each), cut cells in ascending cell order:
 * K [n_cut_stored*36], M [n_cut_stored*36], cut_cells [n_cut_stored]. */
int cb_export_cut_matrices(const cb_ctx* c, double* K, double* M, int64_t* cut_cells);

/* Dense coarse matrix A_c [n_coarse^2] (row-major, host) after cb_factor.
 * Kept for single-problem contexts whose padded coarse matrix fits 1 GiB
 * (n_coarse up to about 11 500); CB_ERR_STATE beyond. */
int cb_export_coarse(const cb_ctx* c, double* Ac);

/* Host-only indexing (no device work): DOF numbering, subdomain sets,
 * objects (Sect. 3.2), variant-1 splitting (Sect. 4.4) and coarse numbering
 * built from given per-cell kept-point counts cell_count [N^3] (> 0 means
 * active), exactly as cb_setup does after its classification kernel.
 * Variant 2 is not available here (it needs the integrated cut cells):
 * CB_ERR_ARG.
 * info receives n_dof, n_sub, n_coarse, n_objects, n_iface; call once with
 * NULL arrays to size them, then again to fill (layouts as in
 * cb_export_indexing).  Errors: CB_ERR_ARG, CB_ERR_SINGULAR. */
int cb_host_indexing(const cb_problem* p, const int32_t* cell_count, cb_info* info, int64_t* dof_node,
                     int32_t* card, int64_t* obj_ptr, int64_t* obj_dofs, int8_t* obj_type,
                     int32_t* coarse_of_obj);

/* Batched SPD inverse building block used by the local and coarse
 * factorisations (blocked Cholesky, triangular inverse, Y^T Y on MFMA):
 * Ainv[b] = A[b]^{-1} for `batch` row-major n x n host matrices, computed on
 * the device in FP64 (precision 0) or FP32 (precision 1).  Synchronous; the
 * default stream.  CB_ERR_NOT_SPD if a pivot is not positive. */
int cb_dense_spd_inverse(int32_t n, int32_t batch, int32_t precision, const double* A, double* Ainv);

/* Allocation-free variant of cb_dense_spd_inverse, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, result and errors; the
 * host arrays A and Ainv are still the caller's.  Every intermediate lives
 * in a fixed 64 MiB device array that the library holds on each GPU it runs
 * on until the process ends: the padded matrices need
 *   batch * (n^2 * 8 + np^2 * (3 s + 8) + ceil(np/128) * 128^2 * s) bytes
 * plus a few KB, np = n rounded up to 32, s = 8 (precision 0) or 4
 * (precision 1), each part rounded up to 256 bytes.  Larger requests return
 * CB_ERR_ARG.  No hipMalloc, hipFree or tuning allocation happens: GEMM tile
 * shapes not tuned before fall back to the default tile.  Calls on one GPU
 * share that array: calls that overlap in time on one GPU race and must be
 * serialised by the caller. */
int cb_dense_spd_inverse_noalloc(int32_t n, int32_t batch, int32_t precision, const double* A, double* Ainv);

const char* cb_last_error(void);
void cb_destroy(cb_ctx* c);

#ifdef __cplusplus
}
#endif
#endif /* CUTBDDC_H */

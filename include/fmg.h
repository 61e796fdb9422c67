/*
 * fmg.h -- C ABI of the MI355X full-multigrid solver for semilinear elliptic
 * problems (Xie & Xu, "A Full Multigrid Method for Semilinear Elliptic
 * Equation").
 *
 * Problem (Section 2, eqs. "semilinear equation", "weak_form", "FEM_form"):
 *     find u_h in V_h with  a(u_h, v) + (f(u_h), v) = (g, v)  for all v in V_h,
 *     a(u, v) = (grad u, grad v),  Omega = (0,1)^dim,  u = 0 on the boundary,
 * V_h = continuous P1 functions (eq. "linear_fe_space") on a mesh of the unit
 * square (right triangles, diagonal from (0,0) to (1,1)) or the unit cube
 * (Kuhn split: six tetrahedra per cube sharing the main diagonal), obtained by
 * `refinements` uniform refinements (beta = 2, eq. "mesh_size_recur") of a
 * coarse grid of `coarse_cells`^dim cells.  The coarse grid is the space V_H
 * of the augmented problems and the first level of Algorithm 3.2.
 * The L2 pairings use the vertex (nodal) quadrature rule on every space.
 *
 * Method (Section 3): Algorithm 3.2 (full multigrid scheme) built on
 * Algorithm 3.1 (one correction step): m V-cycles on the linearised problem
 * (eq. "linearized") from the current iterate, then a small Newton solve on
 * V_H + span{u~} (eq. "coarse problem") whose coefficients are fine-grid
 * quadratures computed on the device.
 *
 * Memory: the caller owns every device buffer (workspace, load, solution,
 * report) and the stream; the library never frees caller memory and makes
 * no device allocation of its own except the hipGraph it may instantiate.
 * All device arrays are float64 nodal arrays of (n+1)^dim entries, x varying
 * fastest, n = coarse_cells * 2^refinements.
 *
 * Errors: argument and size errors are returned synchronously with nothing
 * enqueued.  Numerical outcomes (Newton cap reached, non-finite values) are
 * written by the device into the report.  Calls are stream-ordered and
 * asynchronous unless stated otherwise.  Distinct hierarchies may be used
 * from different threads; one hierarchy must not be used concurrently.
 */
#ifndef FMG_H
#define FMG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FMG_MAX_LEVELS 16

typedef struct fmg_hierarchy fmg_hierarchy;   /* opaque */

enum fmg_status {
    FMG_OK = 0,
    FMG_E_INVALID = 1,        /* null pointer, bad option value            */
    FMG_E_UNSUPPORTED = 2,    /* dim not 2/3, depth out of range, ...      */
    FMG_E_WORKSPACE = 3,      /* workspace too small or misaligned         */
    FMG_E_HIP = 4,            /* a HIP runtime call failed                 */
    FMG_E_NOT_CONVERGED = 5,  /* Newton cap hit (report) / converged mode  */
    FMG_E_NONFINITE = 6,      /* NaN or Inf in the solution (report)       */
    FMG_E_SCRATCH = 7         /* fmg_solve_noalloc: problem needs more than
                                 FMG_NOALLOC_SCRATCH_BYTES of workspace    */
};

/* Nonlinearity catalogue f(u); every entry is nondecreasing (Assumption A). */
enum fmg_nonlinearity {
    FMG_F_ZERO = 0,           /* f = 0                                      */
    FMG_F_LINEAR = 1,         /* f = c u, c = param >= 0                    */
    FMG_F_CUBIC = 2,          /* f = u^3 (Example 1)                        */
    FMG_F_U_PLUS_SIN = 3,     /* f = u + sin u                              */
    FMG_F_ABS_U_U = 4,        /* f = |u| u                                  */
    FMG_F_SIGNED_POW = 5,     /* f = sign(u)|u|^q, q = param >= 1 (Ex. 3)   */
    FMG_F_NEG_EXP = 6         /* f = -exp(-u) (Example 2)                   */
};

enum fmg_precision { FMG_FP64 = 0, FMG_MIXED = 1 };
enum fmg_smoother { FMG_SMOOTHER_DEFAULT = 0, FMG_JACOBI = 1, FMG_CHEBYSHEV = 2 };
enum fmg_mode { FMG_PAPER = 0, FMG_CONVERGED = 1 };
enum fmg_quadrature { FMG_QUAD_VERTEX = 0, FMG_QUAD_ELEMENT = 1 };
enum fmg_coefficients { FMG_COEF_IDENTITY = 0, FMG_COEF_VARIABLE = 1 };

typedef struct {
    int dim;            /* 2 or 3                                           */
    int coarse_cells;   /* cells per side of the coarse grid, >= 2          */
    int refinements;    /* number of uniform refinements, 1..12 (2D), 1..8 (3D) */
} fmg_mesh_desc;

typedef struct {
    int precision;      /* FMG_FP64, or FMG_MIXED: V-cycles in float32 inside
                           float64 residual/update refinement                */
    int m_vcycles;      /* m of Algorithm 3.1 (Section 4: m = 2)             */
    int p_steps;        /* p of Algorithm 3.2 (Section 4: p = 1)             */
    int nu_pre;         /* pre-smoothing sweeps per level                    */
    int nu_post;        /* post-smoothing sweeps per level                   */
    int smoother;       /* FMG_JACOBI (weight omega every sweep) or
                           FMG_CHEBYSHEV (Chebyshev weights on [cheb_lo,
                           cheb_hi] for D^{-1}A, reversed after the coarse
                           correction); DEFAULT = Jacobi 2D, Chebyshev 3D    */
    double omega;       /* Jacobi weight; 0 = 4/5 (2D) or 6/7 (3D)           */
    double cheb_lo, cheb_hi;   /* default 1/3 and 2                          */
    int newton_max;     /* cap on Newton iterations per small solve (30)     */
    double newton_tol;  /* stop when a Newton direction (applied in full) or
                           an accepted damped step d has
                           |d|_inf <= tol max(1,|y|_inf) (1e-14)            */
    int newton_passes;  /* fine quadrature passes per correction step kept in
                           the launch sequence, the setup pass included (3);
                           the last one completes, in one workgroup, any
                           Newton solve that needs more                      */
    int mode;           /* FMG_PAPER: Algorithm 3.2 as stated; FMG_CONVERGED:
                           then repeat correction steps on the finest level
                           until ||du||_2 <= converged_tol ||u||_2 (synchronous).
                           A stop because ||du|| no longer shrinks counts as
                           converged only if ||du||/||u|| <= 1e3 converged_tol;
                           otherwise the report says FMG_E_NOT_CONVERGED */
    int converged_max_steps;
    double converged_tol;
    int use_graph;      /* 1: capture the solve once into a hipGraph and replay */
    int tail_max_nodes; /* V-cycle levels with at most this many interior nodes
                           run together in one launch (0: off): if the top such
                           level has at most 1024, the cycle from it is applied
                           as a dense float64 matrix built at creation (one
                           wavefront per row); otherwise as one single-workgroup
                           recursive cycle with the levels in LDS              */
    int fuse_small_levels; /* 1: run Algorithm 3.2 on those small levels (all
                              steps, incl. the Newton solves) in one launch */
    int aug_max_blocks; /* size of a fine quadrature pass of the augmented
                           problem, in 256-thread workgroups (upper bound;
                           64..16384; 512); large levels run 1024-thread
                           (2D) or 512-thread (3D) workgroups, fewer of them */
    int aug_small_nodes; /* levels with at most this many interior nodes solve
                            the augmented problem in one single-workgroup
                            launch (0: never; default 4096 in 2D, 343 in 3D) */
    int sweep_rows;     /* 2D V(2,2) levels: rows marched by each wavefront of
                           the register-streaming level kernels (2..4096);
                           0 = chosen per level; -1 = LDS-tiled kernels.
                           3D V(2,2) levels with n >= 16: 0 = each sweep pair
                           (pre-smoothing; correction + post-smoothing) in one
                           plane-marching launch; -1 = one launch per sweep,
                           one node per thread; > 0 = one plane-marching
                           launch per sweep                                  */
    int quadrature;     /* FMG_QUAD_VERTEX (default): the L2 pairings (f(u),v)
                           and (g,v) of eq. "FEM_form" and of the augmented
                           problem by the vertex rule, m_j w(x_j);
                           FMG_QUAD_ELEMENT: on every fine simplex a symmetric
                           degree-2 rule (3 points per triangle, 4 per
                           tetrahedron) with u_h, v_h and g as P1
                           interpolants, used everywhere (linearised load,
                           augmented problem, level 1).  Element mode ignores
                           aug_small_nodes and rejects fuse_small_levels = 1
                           and fmg_solve_noalloc with FMG_E_UNSUPPORTED      */
    int coefficients;   /* FMG_COEF_IDENTITY (default): a(u,v) = (grad u,
                           grad v); FMG_COEF_VARIABLE: a(u,v) = (A grad u,
                           grad v) with the symmetric positive definite matrix
                           A(x) of eq. "semilinear equation" constant on every
                           cell of the finest mesh, given by
                           fmg_set_coefficients before the first solve.  Every
                           level carries that one form (Galerkin: the level-k
                           matrix is the finest form on V_{h_k}; on the Kuhn
                           meshes a 7-point (2D) or 15-point (3D) stencil held
                           as per-node edge weights).  Problems may then give
                           f(x,u) = c(x) f(u) (fmg_problem.f_weight).  Needs
                           precision FMG_FP64 and the vertex rule, runs the
                           V-cycles with one-sweep kernels down to level 1 and
                           ignores tail_max_nodes, aug_small_nodes and
                           sweep_rows; fuse_small_levels = 1 and
                           fmg_solve_noalloc return FMG_E_UNSUPPORTED        */
} fmg_options;

typedef struct {
    int kind;               /* enum fmg_nonlinearity                        */
    double param;           /* c (LINEAR) or q (SIGNED_POW)                 */
    const double *g_nodes;  /* device; load g at the finest nodes, (n+1)^dim,
                               boundary entries ignored by the vertex rule
                               (the element rule interpolates g on every
                               simplex, boundary vertices included); must stay
                               valid until the solve has completed on the
                               stream                                        */
    const double *f_weight; /* device or NULL; c(x) >= 0 at the finest nodes,
                               (n+1)^dim, for f(x,u) = c(x) f(u) (vertex
                               rule: m_j c_j f(u_j)); NULL means c = 1.  Only
                               hierarchies with FMG_COEF_VARIABLE take it
                               (else FMG_E_UNSUPPORTED); lifetime as g_nodes  */
} fmg_problem;

typedef struct {
    int status;                          /* enum fmg_status                  */
    int levels;                          /* refinements + 1                  */
    int level1_iters;                    /* Newton iterations on level 1     */
    int extra_steps;                     /* converged mode: extra steps      */
    int newton_iters[FMG_MAX_LEVELS];    /* per level k (index k-1), last step */
    int newton_total[FMG_MAX_LEVELS];    /* per level, summed over the p steps */
    double alpha[FMG_MAX_LEVELS];        /* coefficient of u~ in the last step */
    double last_update_rel;              /* converged mode: ||du|| / ||u||   */
} fmg_report;

/* Fill *opts with the defaults for dimension dim (Section 4: m = 2, p = 1;
 * V(2,2); Jacobi 4/5 in 2D, Chebyshev [1/3, 2] in 3D). */
void fmg_default_options(int dim, fmg_options *opts);

/* Bytes of device workspace fmg_create_hierarchy needs for this mesh and
 * options (0 on invalid input).  Used for admission by memory footprint. */
size_t fmg_workspace_bytes(const fmg_mesh_desc *mesh, const fmg_options *opts);

/* Plan the level hierarchy (Section 3: T_{h_1} .. T_{h_n}, nested spaces,
 * eq. "FEM_Space_Series") inside the caller's workspace d_workspace (device,
 * 256-byte aligned, >= fmg_workspace_bytes bytes, must outlive the
 * hierarchy), upload the level-1 tables and clear the level arrays on
 * `stream` (a hipStream_t).  *out receives the handle. */
int fmg_create_hierarchy(const fmg_mesh_desc *mesh, const fmg_options *opts,
                         void *d_workspace, size_t workspace_bytes, void *stream,
                         fmg_hierarchy **out);

/* FMG_COEF_VARIABLE hierarchies: set the matrix A(x) of the operator
 * -div(A grad u) (Section 2, eq. "semilinear equation"; the form a(u,v) of
 * eq. "weak_form").  d_coef (device, float64) holds the d(d+1)/2 upper-
 * triangle components of A row by row (2D: a11, a12, a22; 3D: a11, a12, a13,
 * a22, a23, a33) as component planes of n^dim cells each (x fastest, a cell
 * named by its lower corner node), A symmetric positive definite per cell;
 * A = kappa I is (kappa, 0, kappa) or (kappa, 0, 0, kappa, 0, kappa).
 * Enqueues on `stream` the kernels that form every level's stencil (the
 * per-simplex means of the finest matrices, the forward edge weights) and
 * the level-1 matrix A_1 and its inverse; d_coef is read by them only, so it
 * may be released once they have completed.  Solves enqueued after this call
 * use the new operator (captured graphs stay valid).  Errors: FMG_E_INVALID
 * (NULL, or a hierarchy created without FMG_COEF_VARIABLE).  Positive
 * definiteness is the caller's: the library does not check it. */
int fmg_set_coefficients(fmg_hierarchy *h, const double *d_coef, void *stream);

/* Solve one problem with Algorithm 3.2.  d_u_out (device, (n+1)^dim float64)
 * receives the finest-level solution with zero boundary.  FMG_COEF_VARIABLE
 * hierarchies return FMG_E_INVALID until fmg_set_coefficients was called.  report may be NULL
 * or point to memory the device can write (device memory or pinned host
 * memory); it is written at the end of the solve.  Asynchronous in FMG_PAPER
 * mode; FMG_CONVERGED mode synchronises the stream once per extra step. */
int fmg_solve(fmg_hierarchy *h, const fmg_problem *prob, double *d_u_out,
              fmg_report *report, void *stream);

/* For callers that cannot allocate device memory (code being captured into a
 * HIP graph, tight serving loops, harnesses that forbid hipMalloc): one solve
 * as fmg_create_hierarchy + fmg_solve + fmg_destroy would do it, with the
 * workspace in a static device buffer of FMG_NOALLOC_SCRATCH_BYTES that the
 * library holds on every GPU it runs on until the process ends, instead of a
 * caller's workspace.  The call allocates nothing on the device or the host
 * heap and captures no graph: it plans on the host stack, clears the level
 * arrays of the buffer, forms the level-1 tables with a kernel and enqueues
 * the solve's kernels on `stream` (asynchronous, stream-ordered).  The
 * caller passes the load, the output d_u_out and (optionally) report exactly
 * as for fmg_solve; the report pointer is the only way to get the status.
 * Differences from the hierarchy path: the small levels of the V-cycle run as
 * a single-workgroup cycle instead of a host-built dense operator (the same
 * operations; results agree to rounding), and only FMG_PAPER mode with the
 * vertex rule and without fuse_small_levels is supported (else
 * FMG_E_UNSUPPORTED).  Sizes: a
 * workspace above FMG_NOALLOC_SCRATCH_BYTES returns FMG_E_SCRATCH with
 * nothing enqueued (2D up to 1024^2 and 3D up to 64^3 fit, both precisions).
 * Every call on a GPU uses that GPU's one buffer, which keeps the last call's
 * contents: calls that overlap on one GPU (two streams, two threads) race and
 * must be serialised by the caller. */
#define FMG_NOALLOC_SCRATCH_BYTES (64u << 20)
int fmg_solve_noalloc(const fmg_mesh_desc *mesh, const fmg_options *opts, const fmg_problem *prob,
                      double *d_u_out, fmg_report *report, void *stream);

/* Copy the report of the last solve to host memory (synchronises `stream`). */
int fmg_get_report(fmg_hierarchy *h, fmg_report *host_report, void *stream);

/* Solve `count` independent problems, each on its own hierarchy (any mix of
 * depths, dimensions and nonlinearities), as ONE graph launch on `stream`:
 * the graph holds one branch per problem (its captured solve), and the
 * branches share no memory, so the device runs them side by side.  The
 * executable graph is cached per list of (hierarchy, nonlinearity) pairs
 * (a few lists are kept; fmg_destroy of a member drops them), so repeated
 * batches over the same hierarchies only update the problem arguments.
 * outs[i] and reports[i] as in fmg_solve (reports may be NULL).
 * Errors: FMG_E_INVALID for NULL arguments, a hierarchy or output listed
 * twice; problem errors as in fmg_solve.  Hierarchies in FMG_CONVERGED mode
 * or without graphs make the call solve the list one after another. */
int fmg_solve_batch(fmg_hierarchy *const *hs, const fmg_problem *probs,
                    double *const *outs, fmg_report *const *reports, int count,
                    void *stream);

/* Release the hierarchy's host state and graphs; never frees caller memory.
 * Waits for the device first (hipDeviceSynchronize), so solves still in
 * flight on h finish before its graphs go; the caller's workspace must stay
 * valid until this call returns. */
int fmg_destroy(fmg_hierarchy *h);

const char *fmg_status_str(int status);

/* Single operators of the multigrid cycle on one level, for verification.
 * Arrays are device float64 (n_k+1)^dim nodal arrays of level `level`
 * (1-based; level n is the finest) except where noted; they are staged
 * through the hierarchy's own level arrays (so no solve may be in flight).
 * precision selects the float64 or float32 kernel instance.
 *   FMG_OP_APPLY_A   out = A_k in0                      (stiffness, Section 2)
 *   FMG_OP_SMOOTH    out = in0 + omega D^{-1}(in1 - A_k in0)   (one sweep)
 *   FMG_OP_RESTRICT  out (level k-1) = P_k^T (in1 - A_k in0)   (residual)
 *   FMG_OP_PROLONG   out = in1 + P_k in0, in0 on level k-1
 *   FMG_OP_COARSE    out = A_1^{-1} in0 (level must be 1)
 * Boundary entries of out are written as zero. */
enum fmg_level_op { FMG_OP_APPLY_A = 0, FMG_OP_SMOOTH = 1, FMG_OP_RESTRICT = 2,
                    FMG_OP_PROLONG = 3, FMG_OP_COARSE = 4 };
int fmg_level_op(fmg_hierarchy *h, int op, int level, int precision,
                 const double *in0, const double *in1, double *out, double omega,
                 void *stream);

/* Diagnostic (measurement): time one of the solve's level kernels on its own.
 * `kernel` is a kernel class as reported by fmg_profile_solve and named by
 * fmg_kernel_name; supported: the fused 2D V(2,2) level kernels
 * ("pre_sweeps_restrict_2d*", "prolong_post_sweeps_2d*", whichever variant
 * the hierarchy's options select), the fused 3D sweep pairs
 * ("pre_sweep_pair_3d_f64/f32", "prolong_sweep_pair_3d_f64/f32"), the 3D
 * plane-marching sweep ("smooth_3d_stream_f64/f32") and the separate sweep
 * ("smooth_f64/f32"), residual-restriction and prolongation-correction
 * kernels, in float64 or (mixed-mode hierarchies) float32; in
 * FMG_COEF_VARIABLE hierarchies the stencil-array sweep and residual
 * ("smooth_var_f64", "resid_var_f64", after fmg_set_coefficients) and the
 * prolongation.  The kernel is
 * launched with the solve's launch shape on level `level` (2..levels) of the
 * hierarchy's own buffers, which it overwrites (no solve may be in flight on
 * `h`): once untimed, then `reps` times back to back on `stream` between two
 * HIP events.  Writes the mean time per launch (ms) and the algorithmic bytes
 * of one launch (each nodal array read or written once).  Synchronises
 * `stream`.  Errors: FMG_E_INVALID (NULL, level or reps out of range),
 * FMG_E_UNSUPPORTED (class not launched this way by this hierarchy). */
int fmg_time_level_kernel(fmg_hierarchy *h, int kernel, int level, int reps,
                          void *stream, double *ms_per_launch,
                          double *bytes_per_launch);

/* Measurement: one solve with plain (uncaptured) launches and a pair of
 * hipEvents recorded on `stream` around every kernel launch.  Entries are
 * aggregated per (kernel class, level): launches, summed milliseconds and
 * the algorithmic bytes the launches must move (minimal HBM streams of the
 * operator, e.g. 24 B per node for a float64 Jacobi sweep).  Synchronous.
 * Kernel classes are named by fmg_kernel_name. */
#define FMG_PROFILE_MAX 512
typedef struct {
    int kernel;            /* kernel class id                                */
    int level;             /* level k (0 when not level-specific)            */
    int launches;
    int nodes;             /* interior nodes of the level                    */
    double ms;             /* summed event time of the launches             */
    double bytes;          /* summed algorithmic bytes                       */
} fmg_profile_entry;
typedef struct {
    int count;
    double total_ms;       /* first to last event of the solve               */
    fmg_profile_entry entries[FMG_PROFILE_MAX];
} fmg_profile;
int fmg_profile_solve(fmg_hierarchy *h, const fmg_problem *prob, double *d_u_out,
                      void *stream, fmg_profile *out);
const char *fmg_kernel_name(int kernel);

#ifdef __cplusplus
}
#endif
#endif /* FMG_H */

/*
 * ietidp.h -- C ABI of the MI355X (gfx950) tree-cotree gauged IETI-DP solver
 * for 3D curl-curl magnetostatics on multi-patch subdomains.
 *
 * The method is the dual-primal isogeometric tearing and interconnecting
 * solver of Mally & Merkel, "On Domain Decomposition for Magnetostatic
 * Problems in 3D" (arXiv 2501.04340).  Section numbers and equation labels
 * below refer to that paper.
 *
 * Conventions for every call:
 *   - Return value 0 on success, a negative IETI_ERR_* code on failure;
 *     ieti_last_error() then returns a thread-local, NUL-terminated message
 *     (valid until the next failing call on the same thread).
 *   - All pointer arguments are host pointers unless the name starts with d_
 *     (device pointers on the handle's GPU).  Input arrays are read during
 *     the call only and remain owned by the caller; the library copies what
 *     it needs.  Output arrays are caller-allocated with the sizes reported by
 *     ieti_get_sizes().
 *   - A handle owns all its device memory and is not thread-safe; distinct
 *     handles may be used from distinct threads.
 *   - Floating-point data is IEEE binary64 unless stated otherwise; integer
 *     maps are exact and identical to any conforming implementation of the
 *     numbering described below.
 */
#ifndef IETIDP_H
#define IETIDP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IETI_ABI_VERSION 2

enum {
  IETI_OK = 0,
  IETI_ERR_INVALID_ARG = -1,      /* bad sizes, version mismatch, NULL pointer */
  IETI_ERR_PARTITION = -2,        /* a subdomain is empty, not connected through patch faces, or not
                                     simply connected (Section 2's assumptions); message names it */
  IETI_ERR_TREE = -3,             /* tree restricted to the Dirichlet boundary is not a tree (Section 3) */
  IETI_ERR_NOT_SPD = -4,          /* non-positive pivot in a local factorisation; message names the subdomain */
  IETI_ERR_BREAKDOWN = -5,        /* PCG breakdown: p^T F p <= 0 */
  IETI_ERR_NOT_CONVERGED = -6,    /* maxit reached; outputs and stats are still filled */
  IETI_ERR_HIP = -7,              /* a HIP runtime call failed */
  IETI_ERR_STATE = -8             /* call order violated (e.g. solve before factor) */
};

enum { IETI_GEOM_BOX = 0, IETI_GEOM_ANNULUS = 1 };
enum { IETI_PREC_FP64 = 0, IETI_PREC_MIXED = 1 };
/* Scaling of the Dirichlet preconditioner's jump operator, B_D = D B
 * (Eq. DirPrec takes D_s = I; the scaled variants follow the rho-scaling of
 * the FETI-DP literature that the paper refers to for heterogeneous
 * coefficients): on each multiplier row joining subdomains k and l,
 * delta_k = rho_l / (rho_k + rho_l) and delta_l = rho_k / (rho_k + rho_l),
 * with rho the diagonal entry of the subdomain's stiffness at the DOF
 * (STIFFNESS), or delta = 1/2 (MULTIPLICITY). */
enum { IETI_SCALE_IDENTITY = 0, IETI_SCALE_STIFFNESS = 1, IETI_SCALE_MULTIPLICITY = 2 };

typedef struct ieti_handle ieti_handle; /* opaque, library-owned */

/* Source current density J (Eq. strongMS).  Called with npts physical
 * points xyz[3*i+0..2] (array of structures) and must write J at each point
 * into out_vec3[3*i+0..2].  Called from the thread that calls
 * ieti_assemble, any number of times, with arbitrary point batches. */
typedef void (*ieti_field_fn)(const double* xyz, int64_t npts, double* out_vec3, void* user);

/* Problem statement (Section 2): a multi-patch domain with patches on a
 * structured P0 x P1 x P2 grid (patch (i,j,k) has index i + P0*(j + P1*k)),
 * curl-conforming B-spline spaces of degree p with n_el elements per patch
 * and direction, the grouping of patches into subdomains, a constant
 * reluctivity per patch, the source J, and n x A = 0 on the whole boundary.
 *   geom_kind  IETI_GEOM_BOX:     geom_params = {x0,x1,y0,y1,z0,z1}, uniform
 *                                 axis-aligned patches.
 *              IETI_GEOM_ANNULUS: direction 0 = azimuth (periodic, P0 equal
 *                                 sectors, each one rational quadratic arc),
 *                                 1 = radius, 2 = height;
 *                                 geom_params = {z0, z1, r_0, ..., r_P1}.
 *   periodic   1 where the patch grid wraps (annulus azimuth), else 0.
 *   degree_p   degree of the H^1 B-splines (curl components have degree p-1
 *              along their own direction), 1 <= p <= 6.
 *   patch_to_subdomain [n_patches] values 0..N_sub-1, every id used.
 *   nu_per_patch       [n_patches], > 0.
 * Non-homogeneous Dirichlet data: the boundary coefficients are the L2
 * projection of the tangential trace of A_D onto the tangential traces of
 * the boundary basis functions (over every boundary patch face, Gauss points
 * as in the volume); the loads are lifted by -K a_D and the boundary values
 * are part of the returned coefficient vector. */
typedef struct {
  int32_t version;             /* must equal IETI_ABI_VERSION */
  int32_t geom_kind;
  int32_t patches[3];
  int32_t periodic[3];
  double geom_params[16];
  int32_t degree_p;
  int32_t n_el;
  const int32_t* patch_to_subdomain;
  const double* nu_per_patch;
  ieti_field_fn J;
  void* J_user;
  ieti_field_fn A_D;           /* Dirichlet data n x A = n x A_D on the whole boundary (a vector
                                  field called like J at boundary points); NULL: n x A = 0 */
  void* A_D_user;
} ieti_problem;

typedef struct {
  int32_t precision;   /* IETI_PREC_FP64, or IETI_PREC_MIXED: FP64 factorisation, FP32 copies of the
                          interface blocks for the inner PCG of an FP64 iterative refinement */
  int32_t tile;        /* factor tile size: 0 = default (64) */
  int32_t ordering;    /* 0 = nested dissection of r_V (default), 1 = natural order */
  int32_t gemv_variant; /* 0 = autotune the interface GEMV launch shape on the first factorisation
                           of the handle (kept afterwards); 1..13 = use shape gemv_variant - 1 */
  int32_t scaling;     /* IETI_SCALE_* of the preconditioner (0 = D_s = I as in the paper) */
  int32_t factor_tune; /* 1 = autotune the factorisation's parameters (deferral thresholds of the
                          tile updates, persistent update workgroups) on the first factorisation of
                          the handle, kept afterwards; a candidate must be over 1% faster to replace
                          the current choice; 0 = the handle's current parameters */
  void* hip_stream;    /* hipStream_t to run on; NULL = the library's own stream */
} ieti_factor_opts;

typedef struct {
  double rtol;               /* stop when ||b - F lambda||_2 <= rtol ||b||_2 */
  int32_t maxit;             /* PCG iteration cap (0 = 1000) */
  int32_t check_every;       /* iterations between host convergence checks (0 = 8) */
  const double* lambda0;     /* host initial multipliers [m_r] or NULL (= 0) */
  int32_t use_graph;         /* 1 = replay PCG iterations from a captured hipGraph */
  int32_t warm_start;        /* 1 = lambda_0 from the network set by ieti_set_warm_start (ignored
                                when lambda0 is given); rejected in favour of lambda_0 = 0 when
                                ||b - F lambda_0|| >= ||b|| or not finite */
} ieti_solve_opts;

typedef struct {
  int64_t n_global;      /* n_g: free (non-Dirichlet, non-tree) global DOFs */
  int64_t n_multipliers; /* m_r */
  int64_t n_primal;      /* n_gp */
  int64_t n_sub;
  int32_t iters;         /* PCG iterations */
  int32_t outer_iters;   /* iterative-refinement steps (MIXED) */
  int32_t status;        /* IETI_OK or IETI_ERR_NOT_CONVERGED */
  int32_t f_applies;     /* applications of the interface operator */
  double rel_residual;   /* ||b - F lambda|| / ||b|| at exit */
  double t_factor_s;     /* device time of ieti_factor */
  double t_solve_s;      /* device time of ieti_solve (rhs + PCG + recovery) */
  double t_pcg_s;        /* device time of the PCG loop */
  double factor_flops;   /* algorithmic flops of the local factorisations */
  double rel_residual0;  /* ||b - F lambda_0|| / ||b|| of the initial multipliers used */
  int32_t warm_start;    /* 1 = network prediction used, -1 = prediction rejected, 0 = not asked */
  int32_t reserved;
  double pcg_bytes;      /* algorithmic bytes moved by the PCG phase (see ieti_problem_stats),
                            summed over the problems; divided by t_pcg_s: the solve phase's
                            algorithmic bandwidth */
} ieti_stats;

/* Per-problem results of the last solve of a handle.  The algorithmic byte
 * model of one application of the interface operator F (Eq. intProb) or of
 * the preconditioner M_D (Eq. DirPrec) with s-byte interface-block entries
 * (s = 8 FP64, 4 FP32) is
 *   M:  s sum_k n_I,k (n_I,k + 1) / 2  +  16 sum_k n_I,k  +  24 m_r
 *   F:  the same  +  16 sum_k n_I,k n_p,k  +  8 n_gp^2
 * (each symmetric interface block's lower triangle once; the interface
 * vectors in and out; three multiplier vectors; the local primal coupling
 * in and out and the coarse factor).  pcg_bytes = sum over the solve's
 * applications of these figures. */
typedef struct {
  int32_t iters;          /* PCG iterations (MIXED: summed over the inner solves) */
  int32_t outer_iters;    /* iterative-refinement steps (MIXED) */
  int32_t status;         /* IETI_OK or IETI_ERR_NOT_CONVERGED */
  int32_t warm_start;     /* as in ieti_stats */
  int32_t f_applies[2];   /* applications of F with [0] FP64, [1] FP32 interface blocks */
  int32_t m_applies[2];   /* applications of M_D, same split */
  double rel_residual;    /* ||b - F lambda|| / ||b|| at exit (FP64 operator) */
  double rel_residual0;   /* of the initial multipliers */
  double block_entries;   /* sum_k n_I,k (n_I,k + 1) / 2 over the problem's subdomains */
  double bytes_F[2];      /* algorithmic bytes of one F application, FP64 / FP32 blocks */
  double bytes_M[2];      /* the same for M_D */
  double pcg_bytes;       /* algorithmic bytes of the last solve's applications */
} ieti_problem_stats;

/* Results of problem prob (0 for a single-problem handle) of the last solve. */
int ieti_get_problem_stats(const ieti_handle* h, int32_t prob, ieti_problem_stats* out);

/* Assemble the problem on the host: spline spaces, Galerkin matrices of
 * Eq. discrMS per subdomain, facets and wire basket (Section 2), edge
 * weights and Kruskal spanning tree (Section 3, Fig. weights), primal DOFs
 * (cotree edges of weight 2), multipliers (Eq. gloDP with redundant
 * constraints removed), and uploads everything to the current HIP device.
 *
 * Numbering (exact, shared by every conforming implementation):
 *   control nodes (I,J,K) on an N0 x N1 x N2 grid, N_d = P_d (n_el+p-1) + 1
 *   (P_d (n_el+p-1) if periodic); edge (d,I,J,K) joins node (I,J,K) to
 *   (I,J,K)+e_d; edge id = off_d + I + E_d0 (J + E_d1 K) with E_dc the number
 *   of positions of direction-d edges along axis c, directions stacked
 *   0,1,2.  Kruskal takes edges in increasing (weight, edge id).  Local DOFs
 *   of a subdomain are its non-Dirichlet, non-tree, non-primal edges in
 *   increasing edge id.  Multiplier rows are the remaining interface edges in
 *   increasing edge id, +1 in the lower and -1 in the higher subdomain. */
int ieti_assemble(const ieti_problem* prob, ieti_handle** out);

/* Batch of n independent problems in one handle: the problems' subdomains,
 * multiplier rows, primal DOFs, patches and output coefficients are
 * concatenated in problem order, so that one factorisation plan and one set
 * of launches (and one captured hipGraph per two PCG iterations) covers all
 * of them.  The coarse problem stays per problem (block diagonal) and every
 * problem runs its own PCG recurrence (own step lengths and stopping test,
 * ||b_p - F_p lambda_p|| <= rtol ||b_p||); a finished problem is frozen while
 * the others go on.  ieti_factor / ieti_solve / ieti_set_coefficients then act
 * on the whole batch; a_out holds the problems' coefficient vectors one after
 * the other, stats report the largest iteration count and residual.
 * ieti_get_maps is not available on a batch handle.  ieti_assemble(p, out) is
 * ieti_assemble_batch(p, 1, out). */
int ieti_assemble_batch(const ieti_problem* probs, int32_t n, ieti_handle** out);

/* Assembly options.  primal = 1: the primal DOFs of Section 3 (every cotree
 * edge of weight 2), as ieti_assemble; primal = 0: no primal DOFs, which makes
 * the local matrices K_rr of subdomains whose remaining DOFs do not pin the
 * gradient kernel singular (Section 3) -- for checking that; an edge of three
 * or more subdomains then gets one multiplier, between its first two
 * subdomains, so the interface problem is not the paper's. */
typedef struct {
  int32_t version;   /* must equal IETI_ABI_VERSION */
  int32_t primal;    /* 1 (default) or 0 */
  int32_t reserved[6];
} ieti_assemble_opts;
int ieti_assemble_ex(const ieti_problem* prob, const ieti_assemble_opts* opts, ieti_handle** out);

/* Batch handle built from n single-problem handles (their assembled
 * systems are copied; the inputs stay valid and independent).  Same as
 * ieti_assemble_batch on the handles' problems, without repeating the
 * assembly. */
int ieti_batch_of(const ieti_handle* const* hs, int32_t n, ieti_handle** out);

/* Per problem p of a handle (any argument may be NULL):
 *   ranges [8 p .. 8 p + 7] = {first output coefficient, n_edges, first
 *   multiplier row, m_r, first primal DOF, n_gp, first subdomain, N_sub},
 *   iters[p] and rel_residual[p] of the last solve. */
int ieti_get_batch_info(const ieti_handle* h, int64_t* ranges, int32_t* iters, double* rel_residual);

/* Local factorisations and coarse setup on the GPU (Section 2.1): for every
 * subdomain one partial Cholesky factorisation of the augmented matrix
 * [K_rr K_rp E_I; K_pr K_pp 0; E_I^T 0 0] eliminating the r block, which
 * yields the Dirichlet-preconditioner Schur complement S_rIrI (Eq. DirPrec),
 * the local inverse block (K_rr^{-1})_{II}, the primal coupling
 * (K_rr^{-1} K_rp)_{I} and the local coarse contribution; then the coarse
 * matrix (minus F of the paper, positive definite) and its Cholesky factor.
 * Returns IETI_ERR_NOT_SPD if a pivot is not positive. */
int ieti_factor(ieti_handle* h, const ieti_factor_opts* opts);

/* Solve the interface problem (Eq. intProb) by PCG with the Dirichlet
 * preconditioner (D_s = I), then recover a_p (Eq. coarseProb) and a_r
 * (Eq. localProb).  a_out: host [n_edges] (every global edge; Dirichlet and
 * tree edges are 0) or NULL.  stats may be NULL. */
int ieti_solve(ieti_handle* h, const ieti_solve_opts* opts, double* a_out, ieti_stats* stats);

/* As ieti_solve, but writes the coefficient vector to device memory
 * d_a_out [n_edges] (e.g. a torch tensor's storage on the same device). */
int ieti_solve_device(ieti_handle* h, const ieti_solve_opts* opts, double* d_a_out, ieti_stats* stats);

/* sizes[0..7] = {n_edges, n_global, sum_n_r, m_r, n_gp, N_sub, n_nodes, max_n_I}
 * (totals over the problems of a batch handle) */
int ieti_get_sizes(const ieti_handle* h, int64_t* sizes);

/* Exact integer maps (any argument may be NULL):
 *   weight       [n_edges]  edge weights 1..5 (Fig. weights)
 *   tree_mask    [n_edges]  1 = tree edge
 *   dirichlet    [n_edges]  1 = Dirichlet edge
 *   primal_edges [n_gp]     global primal edge ids, increasing
 *   mult_rows    [m_r*5]    per row: edge id, k, l, local index in k, local index in l
 *   sub_offsets  [N_sub+1]  offsets into sub_r_edges
 *   sub_r_edges  [sum n_r]  remaining local DOFs of each subdomain (edge ids) */
int ieti_get_maps(const ieti_handle* h, uint8_t* weight, uint8_t* tree_mask, uint8_t* dirichlet,
                  int64_t* primal_edges, int64_t* mult_rows, int64_t* sub_offsets, int64_t* sub_r_edges);

/* Subdomain k's assembled blocks in local numbering (r DOFs, then primal
 * DOFs in increasing edge id) as CSR over the (n_r+n_p) x (n_r+n_p) matrix,
 * and its load vector.  Call first with NULL arrays to get n and nnz. */
int ieti_get_local_system(const ieti_handle* h, int32_t k, int64_t* n, int64_t* nnz,
                          int64_t* indptr, int32_t* indices, double* values, double* load);

/* Device results of ieti_factor for subdomain k (host copies), interface
 * DOFs in multiplier-row order: S [n_I*n_I] the Schur complement S_rIrI,
 * Sinv [n_I*n_I] = (K_rr^{-1})_{II}, both row-major; either may be NULL.
 * n_I_out receives n_I. */
int ieti_get_schur(const ieti_handle* h, int32_t k, int64_t* n_I_out, double* S, double* Sinv);

/* One application q = F lambda of the interface operator (positive definite
 * form, = -S of Eq. intProb) on host vectors [m_r]; for parity tests. */
int ieti_apply_F(ieti_handle* h, const double* lambda, double* q);

/* One application z = M_D^{-1} r of the Dirichlet preconditioner (Eq. DirPrec). */
int ieti_apply_M(ieti_handle* h, const double* r, double* z);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * application q = F lambda as ieti_apply_F, on device vectors d_lambda [m_r]
 * and d_q [m_r] (distinct, caller-owned) and on `hip_stream` (NULL: the
 * handle's stream), with no allocation, copy or synchronisation.  Its work
 * vectors (gathered interface values, local products, GEMV partial sums,
 * coarse projections) live in one fixed device array of
 * IETI_NOALLOC_SCRATCH_BYTES per GPU, created with the library's code object
 * and held until the process ends; a handle whose work vectors do not fit
 * gets IETI_ERR_INVALID_ARG (ieti_apply_F has no such limit).  Every call on
 * a GPU shares that GPU's array: calls that overlap on one GPU (several
 * streams or threads) race, and the caller must serialise them.  The handle
 * must be factored and its device current; the result is returned
 * asynchronously on the stream. */
#define IETI_NOALLOC_SCRATCH_BYTES (32ll << 20)
int ieti_apply_F_noalloc(ieti_handle* h, const double* d_lambda, double* d_q, void* hip_stream);

/* Right-hand side b = e - G S_c^{-1} d of the interface problem [m_r]. */
int ieti_get_rhs(ieti_handle* h, double* b);

/* Parameters of the local factorisations' schedule (Section 2.1, the blocks
 * of K_rr): a target tile's deferred updates are issued once `defer` of them
 * are pending (`defer_tail` inside a subdomain's dense r_I tail) or at the
 * target's deadline; the update launches use at most `update_wgs`
 * persistent workgroups.  Defaults 8, 4, 2048.  Takes effect at the next
 * ieti_factor (a changed threshold rebuilds the plan) and turns that
 * handle's autotuning off.  A subdomain gets the same tasks, and bitwise the
 * same factor, in any batch factored with the same parameters. */
int ieti_set_factor_params(ieti_handle* h, int32_t defer, int32_t defer_tail, int32_t update_wgs);
/* The parameters in use, params[3] = {defer, defer_tail, update_wgs}, and
 * the autotuner's record log [n_log][4] = {defer, defer_tail, update_wgs,
 * milliseconds per local factorisation} (n_log = 0 when it has not run);
 * any output may be NULL. */
int ieti_get_factor_tuning(const ieti_handle* h, int32_t* params, double* log, int32_t* n_log);

/* Factorisation plan statistics, info[0..9] = {tile pool elements, S/Sinv
 * elements, algorithmic flops of the tile factorisation, flops of the same
 * factorisation done densely, sequential steps, update tasks, sum of n_I^2
 * (interface-block entries read per operator application), number of
 * interface slots (padded), max padded n_I, tile size}, info[10..11] = the
 * scalar work sum_j c_j^2 of the Cholesky factorisation in the same
 * elimination order without tiles or padding (c_j: off-diagonal entries of
 * column j of the factor), of K_rr alone (the local factorisations of
 * Section 2.1) and with the augmented trailing rows that yield the explicit
 * interface blocks.  info holds 12 doubles. */
int ieti_get_plan_info(const ieti_handle* h, double* info);

/* Kernel timing for roofline measurements.  enable = 1 clears the counters
 * and records HIP events at the boundaries of every launch of the interface
 * GEMV (operator and preconditioner) and of the tile-update kernel of the
 * factorisation; while enabled, solves launch PCG kernels directly instead of
 * replaying the captured graph.  enable = 0 stops recording. */
int ieti_set_profiling(ieti_handle* h, int32_t enable);

/* Launch shape of the interface GEMV chosen for FP64 (variant[0]) and FP32
 * (variant[1]) blocks, -1 if not chosen yet, and the autotuner's average
 * time in ms of one application with each of the 13 shapes (timed
 * alternating the operator and preconditioner blocks), ms[13 * precision +
 * shape] (0 if not timed).  Shapes 0..11 stream whole rows of the dense
 * blocks: 4 waves of rows_per_wave = {2,4,8}[s / 4] rows, (s / 2) % 2 + 1
 * 16-byte vectors in flight per lane and row, non-temporal loads if s is
 * odd; they give bitwise identical results.  Shape 12 uses the symmetry of
 * the blocks: it reads every lower 64x64 tile once (half the bytes) and
 * sums the transposed contributions through partials, in another (fixed)
 * order.  Either argument may be NULL. */
int ieti_get_gemv_tuning(const ieti_handle* h, int32_t* variant, float* ms);

/* times[0..11] = {FP64 GEMV launches, FP64 GEMV total ms, update launches,
 * update total ms, update tasks executed, FP64 interface-block bytes read per
 * GEMV application with the chosen FP64 shape, the same for the
 * row-streaming shapes (whole padded blocks), the same for the symmetric
 * shape (lower tiles, the entries inside n_I), the algorithmic FP64 bytes of one application
 * (8 sum_k n_I,k (n_I,k + 1) / 2, no padding), FP32 GEMV launches, FP32
 * GEMV total ms, 0}.  With the symmetric shape the GEMV launches and times
 * are those of its tile kernel. */
int ieti_get_kernel_times(const ieti_handle* h, double* times);

/* Change the reluctivity of every patch and scale every patch's load
 * vector without repeating the assembly: the Galerkin matrix of Eq. discrMS
 * is linear in the piecewise-constant reluctivity, so the library keeps the
 * per-patch contributions and re-sums them (bit-identical to assembling with
 * the new reluctivity).  load_scale[q] multiplies the load of patch q, which
 * equals assembling with the source scaled by load_scale[q] on patch q; the
 * caller keeps the scaled source divergence-free (e.g. one factor per coil
 * ring).  nu_per_patch [n_patches] > 0, load_scale [n_patches] finite; either
 * may be NULL to keep the current values.  The next solve needs a new
 * ieti_factor. */
int ieti_set_coefficients(ieti_handle* h, const double* nu_per_patch, const double* load_scale);

/* Record the PCG step lengths alpha_i and direction updates beta_i of the
 * first cap iterations of every problem (device memory of 16 cap bytes per
 * problem, owned by the handle); cap = 0 stops recording and frees it.  The
 * coefficients define the Lanczos tridiagonal of the preconditioned operator
 * (Section 4 estimates the condition number from it): diagonal 1/alpha_i +
 * beta_{i-1}/alpha_{i-1}, off-diagonal sqrt(beta_i)/alpha_i.  Captured
 * launch graphs are rebuilt on the next solve. */
int ieti_record_pcg(ieti_handle* h, int32_t cap);

/* Coefficients of problem prob's last PCG run (in mixed precision: its last
 * inner run): *n_out = min(iterations, cap), alpha[n_out] and beta[n_out]
 * (either may be NULL; beta of an iteration that met the tolerance is 0).
 * IETI_ERR_STATE if recording is off or no solve ran since it was enabled. */
int ieti_get_pcg_coefficients(const ieti_handle* h, int32_t prob, double* alpha, double* beta, int32_t* n_out);

/* Extreme eigenvalues of the Lanczos tridiagonal built from problem prob's
 * recorded PCG coefficients (ieti_get_pcg_coefficients): estimates of the
 * extreme eigenvalues of the preconditioned interface operator, whose ratio
 * is the condition number Section 4 reports.  Computed by bisection on the
 * Sturm sequence of the tridiagonal (Gershgorin bounds, to relative width
 * 1e-15).  1 and 1 when the run took no iteration. */
int ieti_get_condition(const ieti_handle* h, int32_t prob, double* lambda_min, double* lambda_max);

/* Multipliers of the last solve [m_r]. */
int ieti_get_lambda(const ieti_handle* h, double* lambda_out);

void ieti_destroy(ieti_handle* h);

/* ---- learned warm start ---------------------------------------------------
 * A multilayer perceptron, trained on multipliers that the solver itself
 * computed, predicts the initial multipliers lambda_0 of the PCG from the
 * per-patch reluctivity and load scales.  The PCG then runs as before from
 * lambda_0; the stopping test is the same, so a poor prediction costs
 * iterations, not accuracy.
 *
 * Network: n_layers hidden layers of width n_hidden with tanh, a linear
 * output of n_comb * n_out values; the prediction of a row is
 * pred[o] = sum_r c[r] * out[r * n_out + o] with the row's n_comb
 * coefficients c (the solution is linear in the source, so c carries source
 * amplitudes).  Parameters: for each layer l the matrix W'_l = [W_l b_l]
 * (d_l x (d_{l-1} + 1), row-major, bias in the last column), layers in order,
 * FP32.  Training minimises the mean of (pred - target)^2 over rows and
 * outputs with Adam (Kingma & Ba 2015, Algorithm 1) on shuffled minibatches;
 * forward, backward and the update run on the GPU in FP32. */
typedef struct ieti_nn ieti_nn; /* opaque, library-owned, on the current HIP device */

typedef struct {
  int32_t n_in;      /* input features per row, >= 1 */
  int32_t n_hidden;  /* width of every hidden layer, >= 1 */
  int32_t n_layers;  /* hidden layers, >= 1 */
  int32_t n_comb;    /* coefficients per row, >= 1 */
  int32_t n_out;     /* outputs per row, >= 1 */
} ieti_nn_arch;

typedef struct {
  int32_t epochs;    /* passes over the data */
  int32_t batch;     /* rows per Adam step (0 = 256) */
  float lr;          /* step size alpha */
  float beta1;       /* 0 = 0.9 */
  float beta2;       /* 0 = 0.999 */
  float eps;         /* 0 = 1e-8 */
  uint64_t seed;     /* shuffling: Fisher-Yates driven by SplitMix64 (Steele et al. 2014) */
} ieti_nn_train_opts;

/* New network with all parameters 0 (set them with ieti_nn_set_params). */
int ieti_nn_create(const ieti_nn_arch* arch, ieti_nn** out);
int ieti_nn_num_params(const ieti_nn* nn, int64_t* n_params);
/* Copy parameters in / out [n_params]; setting them also resets Adam's state. */
int ieti_nn_set_params(ieti_nn* nn, const float* params);
int ieti_nn_get_params(const ieti_nn* nn, float* params);
/* Training data (host, copied to the device): X [n][n_in], C [n][n_comb],
 * Y [n][n_out] row-major. */
int ieti_nn_set_data(ieti_nn* nn, const float* X, const float* C, const float* Y, int64_t n);
/* Mean squared error over rows [row0, row0 + nrows) of the data and its
 * gradient grad [n_params] (host) at the current parameters. */
int ieti_nn_loss_grad(ieti_nn* nn, int64_t row0, int64_t nrows, double* loss, float* grad);
/* Adam training on the data; epoch_loss [epochs] (mean squared error of the
 * minibatches of each epoch, before their steps) may be NULL. */
int ieti_nn_train(ieti_nn* nn, const ieti_nn_train_opts* opts, double* epoch_loss);
/* pred [n][n_out] for host inputs X [n][n_in], C [n][n_comb]. */
int ieti_nn_predict(ieti_nn* nn, const float* X, const float* C, int64_t n, float* pred);
void ieti_nn_destroy(ieti_nn* nn);
/* Write the architecture, parameters (FP32) and normalisation to a file /
 * create a network on the current device from such a file.  IETI_ERR_INVALID_ARG if the file
 * cannot be opened, is not a network file of this library (tag, sizes and
 * parameter count are checked before any device allocation) or is
 * truncated.  Adam's state is not stored: a loaded network starts afresh. */
int ieti_nn_save(const ieti_nn* nn, const char* path);
int ieti_nn_load(const char* path, ieti_nn** out);

/* Initial parameters: every weight uniform in [-l, l] with
 * l = sqrt(6 / (d_in + d_out)) of its layer (Glorot & Bengio 2010), biases
 * 0, drawn from SplitMix64 (Steele et al. 2014) seeded with `seed` (53-bit
 * uniforms, layers in order, rows of W'_l in order).  Resets Adam's state. */
int ieti_nn_init_params(ieti_nn* nn, uint64_t seed);
/* Input normalisation and output scale of the network: it computes on rows
 * x' = (x - shift) * scale, and its predictions are out_scale times its
 * output.  Training data (ieti_nn_set_data) and prediction inputs are raw
 * rows; the targets are divided by out_scale for training, so loss and
 * gradient are in the normalised coordinates.  A new network has the
 * identity (shift 0, scale 1, out_scale 1); NULL arrays set the identity.
 * Set it before ieti_nn_set_data. */
int ieti_nn_set_normalisation(ieti_nn* nn, const float* shift, const float* scale, double out_scale);
/* Normalisation fitted to rows X [n][n_in], Y [n][n_out]: shift = column
 * means of X, scale = 1 / column standard deviation (1 where it is below
 * 1e-12), out_scale = root mean square of Y (1 if 0). */
int ieti_nn_fit_normalisation(ieti_nn* nn, const float* X, const float* Y, int64_t n);
int ieti_nn_get_normalisation(const ieti_nn* nn, float* shift, float* scale, double* out_scale);
/* Training rows in a file: appended to `path` (created with a header of
 * the three row sizes on first use; rows of other sizes are rejected). */
int ieti_nn_dataset_append(const char* path, const float* X, const float* C, const float* Y, int64_t n,
                           int32_t n_in, int32_t n_comb, int32_t n_out);
/* Train a network of architecture `arch` on every row of a dataset file:
 * parameters from ieti_nn_init_params(opts->seed), normalisation fitted to
 * the rows, Adam with `opts`, then written to `model_out` (ieti_nn_save).
 * epoch_loss [opts->epochs] may be NULL. */
int ieti_nn_train_file(const char* dataset_path, const ieti_nn_arch* arch, const ieti_nn_train_opts* opts,
                       const char* model_out, double* epoch_loss);

/* How the solver forms the network's rows and places its predictions: one
 * row per facet f (e.g. one interface facet of two subdomains), features
 * x[j] = log(nu[feat_patch[f][j]]) (normalised by the network),
 * coefficients c[r] = load_scale[comb_patch[f][r]], and
 * lambda_0[out_row[f][o]] = out_sign[f][o] * pred[f][o] with the network's
 * (scaled) prediction (out_row -1 = unused output; rows not covered start
 * at 0).  The training target of output o is out_sign[f][o] times the
 * solved multiplier of row out_row[f][o]. */
typedef struct {
  int32_t n_facets, n_feat, n_comb, n_out;
  const int32_t* feat_patch;   /* [n_facets * n_feat] */
  const int32_t* comb_patch;   /* [n_facets * n_comb] */
  const int32_t* out_row;      /* [n_facets * n_out], distinct rows in [0, m_r) or -1 */
  const int8_t* out_sign;      /* [n_facets * n_out], +1 or -1 */
} ieti_warm_layout;

/* Attach a copy of the network's current parameters and normalisation and
 * the layout to the handle (nn may be destroyed afterwards); solves with
 * warm_start = 1 then predict lambda_0 on the GPU. */
int ieti_set_warm_start(ieti_handle* h, const ieti_nn* nn, const ieti_warm_layout* layout);
/* The network's rows for the handle's current coefficients: X [n_facets][n_feat]
 * raw features, C [n_facets][n_comb], and Y [n_facets][n_out] the targets
 * from the multipliers of the last solve (IETI_ERR_STATE before a solve).
 * Any of X, C, Y may be NULL. */
int ieti_warm_rows(const ieti_handle* h, const ieti_warm_layout* layout, float* X, float* C, float* Y);
/* ieti_warm_rows of the last solve appended to a dataset file
 * (ieti_nn_dataset_append): the solver generating its own training data. */
int ieti_warm_append(const ieti_handle* h, const ieti_warm_layout* layout, const char* dataset_path);
/* Load a network file (ieti_nn_load) and attach it (ieti_set_warm_start). */
int ieti_warm_load(ieti_handle* h, const char* model_path, const ieti_warm_layout* layout);
/* The initial multipliers the attached network predicts for the handle's
 * current coefficients, host lambda0 [m_r] (the warm start's lambda_0
 * before its residual check). */
int ieti_warm_predict(ieti_handle* h, double* lambda0);

const char* ieti_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* IETIDP_H */

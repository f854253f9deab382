/* connreg.h -- C ABI of libconnreg, the MI355X (gfx950) solver for spatial
 * connectome regression by the greedy rank-one ALS + Galerkin method of
 * Kuerschner, Dolgov, Harris & Benner, "Greedy low-rank algorithm for
 * spatial connectome regression".
 *
 * Problem (eq. obj_fun without the sign constraint):
 *     min_W 1/2 ||P_Omega(W X - Y)||_F^2 + lambda/2 ||L_y W + W L_x^T||_F^2
 * with normal equation (eq. multitermSylv)
 *     A(W) = lambda (W L_x^2 + 2 L_y W L_x + L_y^2 W)
 *            + sum_a diag(Omega_a) W X_a X_a^T  =  D = (Omega o Y) X^T.
 * W (n_y x n_x) is never formed: it is kept as W = U Z V^T.
 *
 * Conventions for every entry point:
 *  - Matrices are column-major with an explicit leading dimension (ld >= rows).
 *  - Pointers marked [dev] are device pointers (HIP global memory, e.g. torch
 *    tensors); [host] are host pointers.  The caller owns every array it
 *    passes; the library never frees caller memory.  The problem handle owns
 *    copies of the problem data and its workspace (allocated at create or on
 *    first use, freed at destroy).
 *  - Work is enqueued on the handle's stream.  Entry points that return host
 *    scalars (norms, statistics) synchronise that stream before returning.
 *  - Return values: CR_OK = 0; negative = hard error, outputs undefined, a
 *    message is available from cr_last_error(); positive = soft status,
 *    outputs valid (a cap was hit, or a breakdown ended the greedy loop).
 *  - One handle per stream; a handle is not thread-safe.
 */
#ifndef CONNREG_H
#define CONNREG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CR_OK = 0,
  CR_EINVAL = -1,      /* invalid argument (sizes, layout, non-Laplacian input) */
  CR_ENOMEM = -2,      /* device allocation failed                              */
  CR_EHIP = -3,        /* a HIP runtime call failed                             */
  CR_ENONFINITE = -4,  /* NaN/Inf met in inputs or iterates                     */
  CR_NOTCONV = 1,      /* an inner or outer iteration cap was hit               */
  CR_BREAKDOWN = 2,    /* new ALS vector lies in span(U) or span(V): stopped    */
  CR_PC_FALLBACK = 3   /* the learned preconditioner was replaced by Jacobi     */
} cr_status;

typedef enum {
  CR_PREC_FP64 = 0,    /* every vector, product and reduction in FP64            */
  CR_PREC_MIXED = 1    /* FP32 vectors/products with FP64 reductions, FP64
                          Galerkin solve, residual and stopping test             */
} cr_precision;

/* Graph Laplacian L = Deg - Adj of a voxel face-adjacency graph, CSR, [host].
 * Must be symmetric with off-diagonal entries -1, diagonal = number of
 * off-diagonal entries in the row, at most 8 neighbours per voxel; anything
 * else is rejected with CR_EINVAL (the paper's L_x, L_y are such graph
 * Laplacians: section on the mathematical formulation). */
typedef struct {
  int64_t n;
  const int32_t* rowptr;   /* n+1 */
  const int32_t* colidx;   /* rowptr[n] */
  const double* val;       /* rowptr[n] */
} cr_csr;

typedef struct {
  cr_csr Ly;               /* target Laplacian, n_y x n_y                      */
  cr_csr Lx;               /* source Laplacian, n_x x n_x                      */
  int64_t n_inj;           /* number of injections                             */
  const double* X;  int64_t ldx;    /* [dev] n_x x n_inj injection densities   */
  const double* Y;  int64_t ldy;    /* [dev] n_y x n_inj target densities      */
  const uint8_t* Omega; int64_t ldo;/* [dev] n_y x n_inj, 1 = observed (the
                                       paper's convention, not the stored 1-Omega) */
  double lambda;           /* operator lambda (lambda = lambda_bar n_inj / n_x
                              is the caller's choice)                          */
} cr_problem_desc;

typedef struct cr_problem cr_problem;

/* Copies the Laplacians (host) and X, Y, Omega (device) into handle-owned
 * device storage: an ELL neighbour table per Laplacian, Omega as a bitmask
 * plus per-injection lists of unobserved voxels, Omega o Y and X in the
 * working precision.  `hip_stream` is a hipStream_t (NULL = default stream):
 * the handle's work is ordered on it, and X, Y, Omega are read after the work
 * already queued on it has finished (writes from other streams must be complete
 * before the call).  Set-up transfers are staged through pinned host memory on
 * that stream; the call returns when the handle's data is on the device.
 * Errors: CR_EINVAL for bad sizes or a non-graph-Laplacian, CR_ENOMEM, CR_EHIP. */
cr_status cr_problem_create(const cr_problem_desc* desc, cr_precision prec, void* hip_stream,
                            cr_problem** out);
void cr_problem_destroy(cr_problem* p);

/* ||D||_F = ||(Omega o Y) X^T||_F (FP64; synchronises). */
cr_status cr_rhs_norm(cr_problem* p, double* out);

/* Factored application of the operator of eq. multitermSylv to W = U Z V^T,
 * U [dev] n_y x r, Z [dev] r x r, V [dev] n_x x r.  Outputs [dev]:
 *   F (n_y x (2r + n_inj), ldf) = [ L_y U | L_y^2 U | Omega o (U Z H) ],
 *   G (n_x x 2r, ldg)           = [ L_x V | L_x^2 V ],      H = V^T X,
 * so that, with L_x symmetric,
 *   A(U Z V^T) = lambda (U Z G_2^T + 2 F_1 Z G_1^T + F_2 Z V^T) + F_3 X^T.
 * r = 0 is allowed (F = [0 columns | Omega o 0]).  Asynchronous.
 * _f32: the same in FP32 storage (accumulation in FP32 for the products,
 * FP64 for H); requires a handle created with CR_PREC_MIXED or FP64 (both
 * keep FP32 copies of X). */
cr_status cr_op_apply(cr_problem* p, int64_t r, const double* U, int64_t ldu, const double* Z,
                      int64_t ldz, const double* V, int64_t ldv, double* F, int64_t ldf,
                      double* G, int64_t ldg);
cr_status cr_op_apply_f32(cr_problem* p, int64_t r, const float* U, int64_t ldu, const float* Z,
                          int64_t ldz, const float* V, int64_t ldv, float* F, int64_t ldf,
                          float* G, int64_t ldg);

/* The same operator application returned as one factor pair (eq.
 * multitermSylv with every term kept in low-rank form, L_x symmetric):
 *   A(U Z V^T) = F G^T,  k = 3r + n_inj columns,
 *   F [dev] n_y x k (ldf) = [ lambda U | 2 lambda L_y U | lambda L_y^2 U | Omega o (U Z H) ],
 *   G [dev] n_x x k (ldg) = [ L_x^2 V Z^T | L_x V Z^T | V Z^T | X ],   H = V^T X,
 * so the caller needs no lambda or Z arithmetic to use the result.  U, Z, V
 * as for cr_op_apply; r = 0 gives F = [Omega o 0], G = [X].  FP64 on any
 * handle.  Asynchronous; the handle's workspace may grow (allocation).
 * Errors: CR_EINVAL (null pointers, negative r, leading dimensions below the
 * row counts), CR_ENOMEM, CR_EHIP. */
cr_status cr_op_apply_factors(cr_problem* p, int64_t r, const double* U, int64_t ldu,
                              const double* Z, int64_t ldz, const double* V, int64_t ldv,
                              double* F, int64_t ldf, double* G, int64_t ldg);

/* cr_op_apply (FP64) for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, outputs and errors as cr_op_apply; the call
 * itself allocates nothing.  Its workspace (T = Z H and the split-K
 * partials of H = V^T X) is a static 16 MiB device array that each device
 * holds for the life of the process, looked up when a handle is first
 * created on that device.  Limits: r <= 256 and n_inj <= 256, else
 * CR_EINVAL with a message.  Every call on one device uses the same array
 * (no state carries over between calls: all of it is written before it is
 * read), so calls that overlap on one device -- on two streams or two
 * handles -- race; serialise them.  Asynchronous. */
cr_status cr_op_apply_noalloc(cr_problem* p, int64_t r, const double* U, int64_t ldu,
                              const double* Z, int64_t ldz, const double* V, int64_t ldv,
                              double* F, int64_t ldf, double* G, int64_t ldg);

/* Solver options (Algorithm 1 and its sub-solvers).  Obtain defaults from
 * cr_solve_opts_default() and override fields. */
typedef struct {
  int32_t max_rank;        /* Algorithm 1 rank cap r                                  */
  double tau_dW;           /* stop when delta W <= tau_dW (0 = off)                   */
  double tau_res;          /* stop when ||D - A(W)||_F / ||D||_F <= tau_res (0 = off) */
  double als_delta;        /* ALS stop: | ||u_hat||/||v_hat|| - 1 | <= als_delta (0.1) */
  int32_t als_max_sweeps;  /* ALS sweep cap (10)                                      */
  int32_t als_fixed_sweeps;/* > 0: exactly this many sweeps (lockstep comparisons)    */
  double pcg_rtol;         /* inner PCG relative residual (1e-8)                      */
  int32_t pcg_maxit;       /* inner PCG iteration cap (5000)                          */
  double galerkin_rtol;    /* projected CG tolerance; <= 0: tau/2 (tau = tau_res, else tau_dW) */
  int32_t galerkin_maxit;  /* projected CG cap; <= 0: 50 r + 200                      */
  uint64_t seed;           /* SplitMix64 seed of the initial ALS vectors              */
  double orth_tol;         /* breakdown when ||x_perp|| <= orth_tol ||x|| (1e-10)      */
  int32_t pcg_vpt;         /* voxels per thread in the PCG kernel (0 = auto)          */
  int32_t verbose;         /* 1: one line per rank on stderr                          */
} cr_solve_opts;

void cr_solve_opts_default(cr_solve_opts* o);

typedef struct {
  int32_t sweeps;          /* ALS sweeps done                               */
  double delta;            /* last | ||u_hat||/||v_hat|| - 1 |              */
  double unorm, vnorm;     /* last ||u_hat||, ||v_hat||                     */
  int32_t pcg_iters_u;     /* total PCG iterations, u-systems               */
  int32_t pcg_iters_v;     /* total PCG iterations, v-systems               */
  int32_t pcg_notconv;     /* number of inner solves that hit pcg_maxit     */
} cr_als_stats;

/* One rank-1 ALS update (eqs. ALS_linsys and ALS_linsys_v, the inner loop of
 * Algorithm 1) for the residual R = D - A(U Z V^T) of the current iterate
 * (r >= 0 columns; U, V orthonormal is not required here).
 * v_io [dev] n_x: in = initial vector (normalised internally), out = unit v.
 * u_out [dev] n_y: out = unit u.  Inner systems are solved by Jacobi PCG.
 * Synchronises (reads the sweep test).  Soft status CR_NOTCONV when an inner
 * solve hit its cap. */
cr_status cr_als_step(cr_problem* p, int64_t r, const double* U, int64_t ldu, const double* Z,
                      int64_t ldz, const double* V, int64_t ldv, double* v_io, double* u_out,
                      const cr_solve_opts* opts, cr_als_stats* stats);

/* Galerkin refinement (eq. Proj_Sylv): assembles U^T diag(Omega_a) U,
 * V^T X, U^T L_y U, U^T L_y^2 U, V^T L_x V, V^T L_x^2 V, U^T (Omega o Y) from
 * U [dev] n_y x r and V [dev] n_x x r (orthonormal columns expected), then
 * solves the projected equation for Z by matrix-valued CG in FP64 from the
 * warm start Z_io [dev] r x r (ldz) until
 *   ||U^T D V - A_p(Z)||_F <= rtol ||U^T D V||_F   or maxit iterations.
 * Mixed-precision problems run the CG on a BF16 copy of the Gram tensor
 * U^T diag(Omega_a) U inside iterative refinement: every correction step
 * starts from the residual of the FP64 operator, and the stop above is
 * tested on that residual, so the tolerance means the same in both
 * precisions (iters_out then counts the CG steps of all corrections).
 * Z_io out = solution.  iters_out [host] may be NULL.  Synchronises.
 * Soft status CR_NOTCONV when maxit was hit. */
cr_status cr_galerkin_project(cr_problem* p, int64_t r, const double* U, int64_t ldu,
                              const double* V, int64_t ldv, double* Z_io, int64_t ldz,
                              double rtol, int32_t maxit, int32_t* iters_out);

/* FP64 residual norm ||D - A(U Z V^T)||_F and its value relative to ||D||_F,
 * the residual that Algorithm 1 updates after each Galerkin step ("update
 * residual"; the paper stops on delta W, this norm is the added relative-
 * residual stopping test), from the factored residual R = F_R G_R^T with
 * F_R = [Omega o (Y - U Z H) | U | L_y U | L_y^2 U] and
 * G_R = [X | -lambda L_x^2 V Z^T | -2 lambda L_x V Z^T | -lambda V Z^T]
 * via ||R||_F^2 = trace((F_R^T F_R)(G_R^T G_R)).  The Gram form loses about
 * half the digits: its absolute error is near sqrt(eps) ||F_R|| ||G_R||.
 * When that gives a relative residual below 1e-6 (and the factor width
 * k = n_inj + 3r is at most 1024), the norm is recomputed from CholQR2
 * factors F_R = Q_F R_F, G_R = Q_G R_G as ||R_F R_G^T||_F, whose error is
 * near eps ||F_R|| ||G_R||; if the factors' columns are numerically
 * dependent (a Cholesky pivot fails) the Gram value is kept.  The
 * environment variable CONNREG_RESID_QR (read at handle creation) selects
 * 0 = Gram form only, 1 = automatic (default), 2 = CholQR2 always.  The same
 * evaluation is the greedy solve's relres, whose Grams are updated one basis
 * column at a time.  abs_out / rel_out [host].  Synchronises. */
cr_status cr_residual_norm(cr_problem* p, int64_t r, const double* U, int64_t ldu, const double* Z,
                           int64_t ldz, const double* V, int64_t ldv, double* abs_out,
                           double* rel_out);

typedef struct {
  int32_t rank;            /* rank j just completed                         */
  double relres;           /* ||D - A(W_j)||_F / ||D||_F                    */
  double dW;               /* ||W_j - W_{j-1}||_F / ||W_j||_F               */
  double energy;           /* 1/2 <W,A(W)> - <W,D>                          */
  int32_t sweeps;          /* ALS sweeps                                    */
  int32_t pcg_iters;       /* PCG iterations of this rank (u and v)         */
  int32_t galerkin_iters;  /* projected CG iterations                       */
  double seconds;          /* wall time since the solve started             */
  double J;                /* objective of eq. obj_fun at W_j: energy + 1/2 ||Omega o Y||_F^2 */
} cr_rank_info;

typedef struct {
  int32_t rank;            /* final rank                                    */
  double relres, dW;       /* at the final rank                             */
  int64_t pcg_iters;       /* total PCG iterations                          */
  int64_t galerkin_iters;  /* total projected CG iterations                 */
  int32_t pcg_notconv;     /* inner solves that hit their cap               */
  double seconds;          /* wall time of the call                         */
} cr_solve_stats;

typedef void (*cr_rank_cb)(const cr_rank_info* info, void* user);

/* Algorithm 1 (greedy rank-1 ALS + Galerkin) with outer stop on rank,
 * delta W and the relative residual.  U [dev] n_y x max_rank (ld n_y),
 * V [dev] n_x x max_rank (ld n_x), Z [dev] max_rank x max_rank (ld max_rank);
 * on return the leading rank columns hold orthonormal bases and the core.
 * *rank_io [host]: in = rank to resume from (0 = start from W = 0; otherwise
 * U, V, Z hold a previous result whose U, V are orthonormal), out = final
 * rank.  cb (may be NULL) is called after every rank.  Synchronises.
 * Soft statuses: CR_BREAKDOWN (new direction in the span of the basis),
 * CR_NOTCONV (max_rank reached with a tolerance set and not met). */
cr_status cr_greedy_solve(cr_problem* p, const cr_solve_opts* opts, double* U, double* V,
                          double* Z, int64_t* rank_io, cr_solve_stats* stats, cr_rank_cb cb,
                          void* user);

/* Batched masked Grams G_a = U^T diag(Omega_a) U for every injection a, the
 * data term of eq. Proj_Sylv.  U [dev] n_y x r (ldu); G [dev] n_inj blocks of
 * ldg x ldg (ldg >= r), block a at G + a ldg^2, column-major, full symmetric.
 * mode 0: FP64, exact up to summation order (incremental column form, using
 * the unobserved-voxel lists when they are sparse); mode 1: one Khatri-Rao
 * GEMM C[(a,b), alpha] = sum_i U_ia U_ib omega_i,alpha on the BF16 matrix
 * cores with FP32 accumulation (r <= 256), entry error below
 * 2^-8 ||U_a|| ||U_b|| plus FP32 accumulation.  Asynchronous. */
cr_status cr_masked_gram(cr_problem* p, int64_t r, const double* U, int64_t ldu, int32_t mode,
                         double* G, int64_t ldg);

/* ---------------------------------------------------------------------------
 * Post-processing of a solution W = U Z V^T (the analysis steps the paper
 * applies to its solutions).  Arguments as for cr_op_apply (r >= 1); FP64 on
 * any handle; the handle's workspace may grow; synchronise.
 * ------------------------------------------------------------------------- */

/* SVD of the solution (section on the top-view results): Z is not
 * diagonal, so with the SVD of the core Z = Zu diag(s) Zv^T (one-sided Jacobi
 * rotations on the GPU), W = Uh diag(s) Vh^T with Uh = U Zu [dev] n_y x r
 * (lduh), Vh = V Zv [dev] n_x x r (ldvh), s [dev] r, descending; this is the
 * SVD of W when U and V have orthonormal columns (as cr_greedy_solve returns
 * them).  A column of Zu whose singular value is 0 is returned as 0.
 * sweeps_out [host] may be NULL.  CR_NOTCONV if the rotations did not
 * converge in 60 sweeps (outputs then approximate). */
cr_status cr_core_svd(cr_problem* p, int64_t r, const double* U, int64_t ldu, const double* Z,
                      int64_t ldz, const double* V, int64_t ldv, double* Uh, int64_t lduh,
                      double* s, double* Vh, int64_t ldvh, int32_t* sweeps_out);

/* The objective of eq. obj_fun at W = U Z V^T, evaluated directly in FP64
 * (the cost-against-rank curves of the real-data sections):
 * out3 [host] = { J, 1/2 ||P_Omega(W X - Y)||_F^2, lambda/2 ||L_y W + W L_x^T||_F^2 }.
 * The regulariser goes through the Grams of [L_y U | U] and [V Z^T | L_x V Z^T]. */
cr_status cr_objective(cr_problem* p, int64_t r, const double* U, int64_t ldu, const double* Z,
                       int64_t ldz, const double* V, int64_t ldv, double* out3);

/* Statistics over all n_y x n_x entries w of W = U Z V^T, computed tile by
 * tile on the FP64 matrix cores without storing W (section on dropping the
 * nonnegativity constraint: how many entries are negative and how large).
 * sum_sq_neg = ||W - max(0, W)||_F^2, the squared distance to the projection
 * onto the nonnegative orthant; sum_sq = ||W||_F^2. */
typedef struct {
  double entries;          /* n_y n_x                                      */
  double count_neg;        /* number of entries w < 0                      */
  double min, max;         /* smallest and largest entry                   */
  double max_abs;          /* max |w| (the entrywise infinity norm)        */
  double sum_sq;           /* sum of w^2                                   */
  double sum_sq_neg;       /* sum of w^2 over the negative entries         */
} cr_entry_stats_t;
cr_status cr_entry_stats(cr_problem* p, int64_t r, const double* U, int64_t ldu, const double* Z,
                         int64_t ldz, const double* V, int64_t ldv, cr_entry_stats_t* out);

/* ---------------------------------------------------------------------------
 * ALS u-system access and the learned preconditioner.
 *
 * The u half-step of the ALS (eq. ALS_linsys) solves
 *   A_hat u = R v,  A_hat = lambda (L_y^2 + c1 L_y + c0 I) + diag(d),
 *   c1 = 2 v^T L_x v,  c0 = v^T L_x^2 v,  d_i = sum_a Omega_ia (X_a^T v)^2.
 * The paper gives no preconditioner for it (it uses a sparse direct solve);
 * the library offers Jacobi-PCG and, on full-box target grids, flexible CG
 * (Notay's FCG with one stored direction) preconditioned by a small 3-D
 * convolutional network that the library trains on the GPU.  The network
 * never changes the answer: FCG stops on the same FP64 residual test, and
 * any step whose preconditioned residual is not a descent direction
 * (<r, M r> <= 0 or non-finite) falls back to the Jacobi step.
 * ------------------------------------------------------------------------- */

/* Build the u-system of the rank-1 update at W = U Z V^T for a unit vector v
 * [dev] n_x: rhs_out [dev] n_y = R v, d_out [dev] n_y, coef_out [host] 2 =
 * {c1, c0}.  Synchronises.  FP64 handles only (CR_EINVAL otherwise). */
cr_status cr_u_system(cr_problem* p, int64_t r, const double* U, int64_t ldu, const double* Z,
                      int64_t ldz, const double* V, int64_t ldv, const double* v, double* rhs_out,
                      double* d_out, double* coef_out);

typedef struct cr_pc cr_pc;

/* A preconditioner network for an nx x ny x nz box (voxel index
 * x + nx (y + ny z), the numbering of a full-box target Laplacian), with
 * `channels` hidden channels (1..8), weights drawn from SplitMix64(seed)
 * (He-style scaling).  The network lives on the current device and runs on
 * `hip_stream`. */
cr_status cr_pc_create(int32_t nx, int32_t ny, int32_t nz, int32_t channels, uint64_t seed,
                       void* hip_stream, cr_pc** out);
void cr_pc_destroy(cr_pc* pc);
/* number of float parameters; get/set copy them as one host array in layer
 * order (W0, b0, ..., W4, b4; W[co][ci][27], tap k = 9(dz+1) + 3(dy+1) + (dx+1)) */
int64_t cr_pc_num_params(const cr_pc* pc);
cr_status cr_pc_get_params(cr_pc* pc, float* host_out);
cr_status cr_pc_set_params(cr_pc* pc, const float* host_in);
/* forward on an explicit input in [dev] 4 x N float (channel-major) into
 * y [dev] N float; and its vector-Jacobian product for the upstream gradient
 * dy [dev] N float, returned as parameter gradients in grad_host [host]
 * (same order as get_params).  Both synchronise; for checks and tooling. */
cr_status cr_pc_forward(cr_pc* pc, const float* in, float* y);
cr_status cr_pc_vjp(cr_pc* pc, const float* in, const float* dy, float* grad_host);
/* One Adam step on a batch of u-systems of handle p (whose target graph is
 * the pc's box): b, x, d [dev] batch x n_y (x = exact solutions),
 * coef [host] batch x 2 ([2 v^T L_x v, ||L_x v||^2]).  The network refines
 * the base step w of the flexible CG (the spectral solve when
 * cr_problem_set_box was called, else Jacobi) into z = w_n + y with
 * w_n = sqrt(N) w / ||w||; loss = mean over the batch of 1 - cos^2(z, x),
 * the quantity that a scale-invariant preconditioner step can reduce.
 * loss_out [host]. */
cr_status cr_pc_train_step(cr_pc* pc, cr_problem* p, int32_t batch, const double* b,
                           const double* x, const double* d, const double* coef, float lr,
                           double* loss_out);

/* Solve A_hat x = rhs (FP64) for the u-system of eq. ALS_linsys with data
 * diagonal d [dev] n_y and coef [host] = [2 v^T L_x v, ||L_x v||^2]:
 * precond 0 -> persistent Jacobi-PCG; 1 -> flexible CG with the base step
 * (spectral on a box set by cr_problem_set_box, else Jacobi); 2 -> flexible
 * CG with the base step refined by the network pc (pc required).  x_out
 * [dev] n_y (not normalised); iters_out, relres_out, fallbacks_out [host]
 * may be NULL.  Synchronises. */
cr_status cr_u_solve(cr_problem* p, const double* d, const double* coef, const double* rhs,
                     double* x_out, double rtol, int32_t maxit, int32_t precond, cr_pc* pc,
                     int32_t* iters_out, double* relres_out, int32_t* fallbacks_out);

/* Use pc (NULL: none) for the u-systems of cr_greedy_solve / cr_als_step on
 * this handle (full-box targets matching the pc's box; with a mixed handle
 * the flexible CG runs in FP64 on FP64 copies of the system); sets the
 * u-system preconditioner to 2 (pc) or 0 (NULL).  The handle does not own
 * pc.  Jacobi-PCG takes over any u-solve that the flexible CG does not
 * finish. */
cr_status cr_problem_set_pc(cr_problem* p, cr_pc* pc);

/* u-system preconditioner of cr_greedy_solve / cr_als_step: 0 persistent
 * Jacobi-PCG (default), 1 flexible CG with the base step, 2 flexible CG with
 * the base step refined by the network of cr_problem_set_pc.  CR_EINVAL for
 * other values or 2 without a network. */
cr_status cr_problem_set_precond(cr_problem* p, int32_t kind);

/* Declares the target (which 0) or source (which 1) grid a full
 * dims[0] x dims[1] x dims[2] box numbered first axis fastest.  Checks the
 * Laplacian against the box's free-face 7-point Laplacian (CR_EINVAL if it
 * differs) and builds the per-axis DCT-II eigenbases of the path-graph
 * Laplacians.  Target: the base step of the flexible CG becomes the spectral
 * solve w = Q diag(1 / (lambda (mu^2 + 2 b mu + a) + mean(d))) Q^T r, exact
 * for the u-system of eq. ALS_linsys when d is constant.  Source (with
 * precond 1 or 2 and n_inj <= 128): the v-systems of eq. ALS_linsys_v are
 * solved directly by the Sherman-Morrison-Woodbury identity around the
 * spectral solve of lambda (L_x^2 + 2 c L_x + e I), with FP64 residual
 * refinement; a solve that misses its tolerance falls back to Jacobi-PCG.
 * dims [host]. */
cr_status cr_problem_set_box(cr_problem* p, int32_t which, const int32_t* dims);

/* Two-level preconditioner for the v-systems of eq. ALS_linsys_v (the ALS
 * half-step the paper solves with Sherman-Morrison-Woodbury around a sparse
 * direct solve; here Jacobi-PCG, whose iteration count is set by the nearly
 * singular lam (L_x + c I)^2 part).  The source voxels are grouped into
 * aggregates, the cubes of `block` voxels per axis of their integer
 * coordinates coords [host] (n_x x dim, row-major, the numbering of L_x;
 * dim 1..3); M^-1 = D^-1 + P (P^T B_hat P)^-1 P^T with D the Jacobi
 * diagonal and P the normalised aggregate indicator matrix.  The coarse
 * matrix is assembled and inverted on the GPU for every v-system (m
 * aggregates: a few m^3 flops), and each PCG iteration restricts the
 * residual per aggregate and adds the coarse correction (one more grid
 * barrier per iteration).  The answer does not change (same stopping test).
 * which must be 1 (source); block <= 0 switches it off.  Errors: CR_EINVAL
 * (an aggregate above 256 voxels, more than 2048 aggregates, bad dim).
 * Launches whose two-level grid does not fit co-resident use plain
 * Jacobi-PCG. */
cr_status cr_problem_set_coarse(cr_problem* p, int32_t which, const int32_t* coords,
                                int32_t dim, int32_t block);

/* ---------------------------------------------------------------------------
 * Batched solves and autotuning.
 * ------------------------------------------------------------------------- */

/* Runs Algorithm 1 on `count` independent problems concurrently: K worker
 * threads (K = the largest value <= min(count, 16) for which every problem
 * fits) take problems from a queue, largest first; each problem runs on its
 * own handle and stream (distinct handles on distinct streams are
 * required).  While the call runs, each problem's persistent kernels (PCG,
 * projected CG) are limited to the workgroup slots of 3/4 of 1/K of the
 * device's CUs and launched as ordinary kernels with the library's bounded
 * grid barrier, so the grids of K problems fit on the device at once and
 * overlap.  opts, U, V, Z, ranks, stats, statuses are arrays of `count`
 * entries with the meaning of cr_greedy_solve (stats may be NULL).  Returns
 * the first hard error, CR_OK otherwise; per-problem statuses in statuses[]. */
cr_status cr_greedy_solve_batch(int32_t count, cr_problem** probs, const cr_solve_opts* opts,
                                double** U, double** V, double** Z, int64_t* ranks,
                                cr_solve_stats* stats, int32_t* statuses);

/* Autotuner for the PCG grid shape (the stencil tile of the persistent
 * kernels): times 60 iterations of a representative u- and v-system for
 * voxels per thread 1, 2, 4, 8 (those whose grid fits in cu_share CUs;
 * cu_share <= 0: the whole device) and keeps the fastest for later solves
 * with pcg_vpt = 0.  Outputs [host], may be NULL: chosen values and
 * microseconds per iteration.  FP64 and mixed handles (the mixed handle times
 * its FP32 PCG).  Synchronises. */
cr_status cr_autotune_pcg(cr_problem* p, int32_t cu_share, int32_t* vpt_u, int32_t* vpt_v,
                          double* us_u, double* us_v);
/* Set the tuned values directly (e.g. from a cache); 0 = heuristic. */
cr_status cr_problem_set_tuning(cr_problem* p, int32_t vpt_u, int32_t vpt_v);

/* Message of the last hard error on this thread ("" if none). */
const char* cr_last_error(void);

/* Library version string. */
const char* cr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CONNREG_H */

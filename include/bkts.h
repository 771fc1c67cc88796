/*
 * bkts.h -- Block Krylov Time Stepping on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the hot path of the vectorised parallel-in-time integrator of
 * Engwer, Schell and Dreier, "Vectorized Parallel in Time methods for
 * low-order discretizations with application to Porous Media problems"
 * (arXiv 2504.02117).  Several consecutive implicit time steps (or DIRK
 * stages) of M y' + K y = b (Sec. 1, eq. problem) are collected as the k
 * columns of an N x k block Y and solved together as the matrix equation of
 * Sec. 2.1 with a block Krylov method.
 *
 * Conventions shared by every call:
 *  - Block vectors are ROW-MAJOR N x k arrays with leading dimension ld >= k
 *    (element (r, c) at p[r*ld + c]); they live in device memory (HBM) unless
 *    a parameter says "host".  torch's contiguous (N, k) tensors qualify.
 *  - The caller owns every data pointer.  The library owns only the handles it
 *    creates (ctx, op, tc, nlop, server) and the device workspace behind them;
 *    each handle has a *_destroy call.
 *  - All device work is enqueued on the context's stream, in order.  Calls
 *    that return values to the host (norms, iteration counts, exported arrays)
 *    synchronise that stream before returning; the others are asynchronous.
 *  - Every call returns a bkts_status.  On failure the message is available
 *    from bkts_last_error() (thread-local, valid until the next failing call
 *    on the same thread).  Shapes are validated before any launch: k < 1,
 *    k > BKTS_MAX_K, ld < k, N mismatches or NULL pointers return BKTS_EINVAL
 *    and enqueue nothing.  HIP runtime errors return BKTS_EDEVICE.  No C++
 *    exception crosses this boundary.
 *  - One context per host thread.  Handles must be used with the context that
 *    created them.
 *  - The mass matrix is the identity: every operator built here is scaled per
 *    unit cell volume.
 */
#ifndef BKTS_H
#define BKTS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BKTS_MAX_K 32

typedef enum bkts_status {
  BKTS_OK = 0,
  BKTS_EINVAL = -1,      /* invalid argument or shape; nothing was enqueued     */
  BKTS_ENOMEM = -2,      /* device or host allocation failed                   */
  BKTS_EDEVICE = -3,     /* HIP runtime error                                  */
  BKTS_EBREAKDOWN = -4,  /* Krylov breakdown that deflation could not absorb   */
  BKTS_ENOCONV = -5,     /* iteration limit reached; outputs hold the last iterate */
  BKTS_EBUSY = -6        /* resource temporarily full (server admission)       */
} bkts_status;

typedef struct bkts_ctx_s* bkts_ctx;
typedef struct bkts_op_s* bkts_op;
typedef struct bkts_tc_s* bkts_tc;
typedef struct bkts_nlop_s* bkts_nlop;
typedef struct bkts_server_s* bkts_server;

/* element types of block vectors */
enum { BKTS_F64 = 0, BKTS_F32 = 1 };
/* sparse storage formats of an operator */
enum { BKTS_FMT_CSR = 0, BKTS_FMT_SELL = 1, BKTS_FMT_STENCIL = 2 };

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device`.  `hip_stream` is an existing
 * hipStream_t to enqueue on (e.g. torch.cuda.current_stream().cuda_stream) or
 * NULL for the null stream.  The stream is borrowed, never destroyed. */
bkts_status bkts_ctx_create(int device, void* hip_stream, bkts_ctx* out);
void bkts_ctx_destroy(bkts_ctx ctx);
/* Block until all work enqueued through `ctx` has finished. */
bkts_status bkts_ctx_synchronize(bkts_ctx ctx);
/* Thread-local message of the last failing call ("" if none). */
const char* bkts_last_error(void);
const char* bkts_version(void);

/* Per-kernel device timers.  When enabled, timed launches of the kernels below
 * carry HIP events in their dispatch (the interval is the kernel's own
 * execution), and their algorithmic bytes (the traffic the kernel must move by
 * its definition, e.g. for the block operator nnz*(s+4) + 4(N+1) + 2*N*k*s with
 * s the element size) are accumulated.  bkts_profile_enable(ctx, n) resets the
 * counters and times every launch (n = 1) or every n-th launch of each kernel
 * id (n > 1, to keep the event overhead off the host path); n = 0 disables.
 * bkts_profile_query synchronises and returns the totals over the timed
 * launches of one kernel id. */
enum {
  BKTS_K_SPMM = 0,       /* block operator Y = aX + bKX                      */
  BKTS_K_GRAM = 1,       /* X^T Y                                             */
  BKTS_K_NORMS = 2,      /* column norms                                      */
  BKTS_K_CG_UPDATE = 3,  /* X += P a, R -= Q a with Gram epilogues            */
  BKTS_K_CG_PUPDATE = 4, /* P = D^-1 R + P b                                  */
  BKTS_K_RESIDUAL = 5,   /* fused all-at-once residual                        */
  BKTS_K_SMALL = 6,      /* k x k device kernels and partial-sum folding      */
  BKTS_K_CAST = 7,       /* precision casts / strided copies                  */
  BKTS_K_OTHER = 8,      /* vector helpers of the time-stepping loop          */
  BKTS_K_MG_RESTRICT = 9,  /* multigrid, finest level: smoothed residual restricted */
  BKTS_K_MG_PROLONG = 10,  /* multigrid, finest level: prolongation and post-sweep  */
  BKTS_K_MG_COARSE = 11,   /* multigrid: every coarser level and the coarsest solve */
  BKTS_K_COUNT = 12
};
bkts_status bkts_profile_enable(bkts_ctx ctx, int enable);
bkts_status bkts_profile_query(bkts_ctx ctx, int kernel, int64_t* launches, double* total_ms,
                               double* algorithmic_bytes);
/* The individual durations (ms) of the timed launches of one kernel id since
 * profiling was enabled, in launch order: copies min(total, max) of them into ms
 * and stores the total count in *n (max = 0 and ms = NULL query the count).  A
 * robust statistic (the median) of these is what a benchmark should report for
 * short kernels, whose event intervals occasionally include queue stalls.
 * Synchronises the ctx stream. */
bkts_status bkts_profile_samples(bkts_ctx ctx, int kernel, float* ms, int max, int* n);

/* ---------------------------------------------------------------- operators */

typedef struct bkts_grid {
  int dim;   /* 1, 2 or 3 */
  int n[3];  /* cells per axis, x first; unused axes ignored.  Unit square/cube, h_d = 1/n_d.
                Linear cell index ix + n0*iy + n0*n1*iz. */
} bkts_grid;

enum { BKTS_BC_DIRICHLET = 0, BKTS_BC_NEUMANN = 1 };

typedef struct bkts_fv_coeffs {
  const double* kappa;   /* device, one diffusion coefficient per cell, or NULL: use kappa_const */
  double kappa_const;
  double velocity[3];    /* constant convection velocity (first-order upwind) */
  int bc_type[6];        /* face 2*axis + side (side 0 = low): BKTS_BC_DIRICHLET or BKTS_BC_NEUMANN */
  double bc_value[6];    /* Dirichlet value g of each face */
} bkts_fv_coeffs;

/* Assemble the cell-centred finite-volume operator K and source b of
 * u_t + div(v u - kappa grad u) = 0 (Sec. 4.1 uses a cell-centred FV scheme;
 * the fluxes are this library's reading): interior faces carry the harmonic
 * mean 2 kP kQ / (kP + kQ) / h^2, Dirichlet faces 2 kP / h^2 with b += 2 kP g / h^2,
 * convection is first-order upwind (boundary inflow moves w g / h into b).
 * Runs on the device from the device array `kappa`.  `format` selects the
 * storage used by the block operator (CSR is always kept for export):
 * BKTS_FMT_CSR, BKTS_FMT_SELL (SELL-C, C = 64), or BKTS_FMT_STENCIL, the
 * block operator of Sec. 3 without its column-index stream: with rows numbered
 * as above, every off-diagonal entry sits at an offset s in {1, n0, n0*n1}, and
 * a symmetric K is stored as its diagonal plus one array per offset,
 * o_s[r] = K[r][r+s] = K[r+s][r] ((1 + dim) N values against nnz values and
 * nnz indices).  The block operator, the fused SpMM + Gram of block CG and the
 * fused residual read it; CSR and SELL are kept beside it for export and for
 * the kernels without a stencil variant.  The stencil format needs a symmetric
 * operator: BKTS_EINVAL when a velocity is nonzero (upwind convection).
 * bkts_op_create_csr rejects it (no grid).  It is also what the multigrid
 * preconditioner (BKTS_PREC_MG) is built from. */
bkts_status bkts_fv_assemble(bkts_ctx ctx, const bkts_grid* grid, const bkts_fv_coeffs* coeffs,
                             int format, bkts_op* out);

/* Wrap a caller-provided square CSR matrix (device arrays, int32 indices,
 * sorted or unsorted columns, no duplicates required) as an operator.  The
 * library copies the arrays; the source vector b is zero. */
bkts_status bkts_op_create_csr(bkts_ctx ctx, int64_t N, int64_t nnz, const int32_t* rowptr,
                               const int32_t* col, const double* val, int format, bkts_op* out);
bkts_status bkts_op_info(bkts_op op, int64_t* N, int64_t* nnz);
/* Copy the CSR arrays and source b to HOST buffers (sizes N+1, nnz, nnz, N; any may be NULL).
 * Synchronises. */
bkts_status bkts_op_export_csr(bkts_op op, int32_t* rowptr, int32_t* col, double* val, double* b);
void bkts_op_destroy(bkts_op op);

/* Block operator ("BOP", Sec. 3): Y = alpha * X + beta * K X for N x k blocks
 * of element type `dtype` (BKTS_F64, or BKTS_F32 with FP32 matrix values and
 * FP32 accumulation).  Each matrix entry is read once per block of k columns. */
bkts_status bkts_spmm(bkts_ctx ctx, bkts_op op, int dtype, int k, double alpha, double beta,
                      const void* X, int ldx, void* Y, int ldy);

/* One multigrid V-cycle Z = B F for A = a I + b K, the preconditioner BKTS_PREC_MG
 * applies in every block-CG iteration (Sec. 4.1 preconditions the inner solves
 * with AMG; this is a geometric counterpart).  Galerkin 2x2x2 aggregation of the
 * stencil form of K (and of the identity mass), one damped Jacobi sweep (w = 0.8)
 * before the restriction and one after the prolongation, 12 sweeps on the coarsest
 * level (at most 64 cells).  B is symmetric positive definite.  F, Z: device N x k
 * blocks of type `dtype`, contiguous (ldf = ldz = k), 16-byte aligned, not
 * overlapping (else BKTS_EINVAL).  The op must
 * carry the stencil form (BKTS_FMT_STENCIL), else BKTS_EINVAL; the hierarchy is
 * built on first use and kept with the op. */
bkts_status bkts_mg_apply(bkts_ctx ctx, bkts_op op, int dtype, int k, double a, double b, const void* F,
                          int ldf, void* Z, int ldz);

/* Gram matrix G = X^T Y (k x k, row-major, FP64, DEVICE pointer) of two N x k
 * blocks of type `dtype`, accumulated in FP64 in a fixed order (bitwise
 * reproducible). */
bkts_status bkts_gram(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, int ldx,
                      const void* Y, int ldy, double* G);

/* Allocation-free variant of bkts_gram, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, checks and result as bkts_gram (FP64 accumulation in a
 * fixed order; the fold may differ from bkts_gram's in the last bits).  The
 * per-workgroup partials live in a fixed 4 MiB device array of the library (one
 * copy per GPU, held until the process ends; its address is recorded when a
 * context is created on that GPU), and the number of partials is capped to fit it,
 * so every N is accepted; a fit failure would return BKTS_EINVAL.  The call
 * enqueues two kernels on the ctx stream and calls no allocator.  Calls that
 * overlap on one GPU (other contexts or streams) share the array and race. */
bkts_status bkts_gram_noalloc(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, int ldx,
                              const void* Y, int ldy, double* G);

/* ------------------------------------------------------------ time coupling */

enum { BKTS_IE = 0, BKTS_THETA = 1, BKTS_SDIRK2 = 2, BKTS_DIRK_CUSTOM = 3, BKTS_RADAU2 = 4 };

typedef struct bkts_tc_desc {
  int method;        /* BKTS_IE, BKTS_THETA, BKTS_SDIRK2, BKTS_RADAU2 or BKTS_DIRK_CUSTOM */
  double theta;      /* BKTS_THETA only */
  int stages;        /* BKTS_DIRK_CUSTOM: number of stages m (<= 8) */
  const double* A;   /* BKTS_DIRK_CUSTOM: host, m x m row-major, stiffly accurate (b = last row);
                        lower triangular (DIRK) or full (fully implicit) */
  const double* c;   /* BKTS_DIRK_CUSTOM: host, m; must be the row sums of A with c_m = 1
                        (a consistent stiffly accurate method), else BKTS_EINVAL */
  int k;             /* block width: number of stage columns in one window (1..BKTS_MAX_K) */
  double tau;        /* time step */
} bkts_tc_desc;

/* Build the time coupling of a stiffly accurate Runge-Kutta method (Sec. 2, eq.
 * stiffly-accurate-DIRK; b = last row of A).  A first stage with a zero row
 * is eliminated (Sec. 2.1).  The theta method is the 2-stage scheme
 * [[0,0],[1-theta,theta]]; SDIRK2 is the L-stable 2-stage SDIRK with
 * gamma = 1 - 1/sqrt(2); RADAU2 is the 2-stage Radau IIA method
 * [[5/12,-1/12],[3/4,1/4]], c = (1/3, 1).
 * Fully implicit tableaux (an entry above the diagonal of the implicit part; the
 * remark on fully implicit Runge-Kutta methods after Algorithm 1): A2 holds full
 * m x m diagonal blocks, k must be a multiple of m, windows start at stage 0
 * (phase 0 only), Algorithm 1 accepts a whole step at a time, and the splitting
 * uses one averaged coefficient beta = |det A|^(1/m) for every stage.  BKTS_EINVAL
 * for a singular fully implicit A or such a k.  The time coupling is a host
 * object: `ctx` may be NULL, and a tc can be used with any context. */
bkts_status bkts_tc_create(bkts_ctx ctx, const bkts_tc_desc* desc, bkts_tc* out);
/* Window matrices of eq. time-stepping-matrices-multiple-parallel-time-steps
 * taken from diagonal index `phase` (Sec. 2.2, pipelining): A1, A2 (HOST,
 * k x k row-major) and beta = A2[0][0] (eq. matrix-splitting; the averaged
 * coefficient for a fully implicit tableau).  `phase` is the
 * implicit-stage index of the front column within its step (0 <= phase < m_impl).
 * Any output may be NULL. */
bkts_status bkts_tc_get(bkts_tc tc, int phase, double* A1, double* A2, double* beta, int* k, int* m_impl);
void bkts_tc_destroy(bkts_tc tc);

/* All-at-once residual (Sec. 2.2; the sign of the F term is read so that it
 * matches the linear system of eq. general-system-time-steps):
 *     R = Y A1^T + (K Y - b 1^T) A2^T - B0,       col_norms2[j] = ||R_j||_2^2
 * for the window matrices of `phase`.  Y, R: device N x k (k = the tc's k).
 * B0: device N x nb0 (the first nb0 window columns; the rest are zero) or
 * NULL.  col_norms2: HOST array of k doubles or NULL (synchronises when given).
 * One fused pass: the sparse product, both right multiplications and the norms. */
bkts_status bkts_residual(bkts_ctx ctx, bkts_op op, bkts_tc tc, int phase, const double* Y, int ldy,
                          const double* B0, int ldb0, int nb0, double* R, int ldr, double* col_norms2);

/* ------------------------------------------------------------- block solve */

enum { BKTS_CG = 0, BKTS_GMRES = 1, BKTS_BICGSTAB = 2 };
/* BKTS_PREC_MG: one symmetric geometric multigrid V-cycle per iteration (Galerkin 2x2x2
 * aggregation of the stencil form, damped Jacobi smoothing).  Block CG, block GMRES and BiCGStab
 * (the last two preconditioned from the right); the operator must carry the stencil form
 * (BKTS_FMT_STENCIL), or be the Newton Jacobian of a nonlinear grid operator, whose V-cycle is
 * built from the stencil form of its symmetric part (J + J^T) / 2 and rebuilt after each Jacobian
 * assembly.  Otherwise, or with per-column operators, BKTS_EINVAL.  The paper preconditions its
 * inner solves with AMG (Sec. 4.1). */
enum { BKTS_PREC_NONE = 0, BKTS_PREC_JACOBI = 1, BKTS_PREC_MG = 2 };
enum { BKTS_PRECISION_F64 = 0, BKTS_PRECISION_F32_REFINE = 1 };

typedef struct bkts_solve_opts {
  int krylov;        /* BKTS_CG (SPD operators), BKTS_GMRES, BKTS_BICGSTAB */
  int precond;       /* BKTS_PREC_NONE, BKTS_PREC_JACOBI or BKTS_PREC_MG */
  int precision;     /* BKTS_PRECISION_F64, or FP32 Krylov iterations inside an FP64
                        iterative-refinement loop (residuals in FP64) */
  double rtol;       /* per column: stop when ||r_j|| <= rtol * ||b_j - A x0_j|| for every j */
  int maxit;         /* iteration limit (all inner iterations counted) */
  int restart;       /* GMRES: block Krylov dimension per cycle (in blocks) */
  double inner_rtol; /* F32_REFINE: relative reduction per FP32 inner solve (e.g. 1e-4) */
} bkts_solve_opts;

typedef struct bkts_solve_info {
  int iterations;          /* block Krylov iterations (one block operator application each) */
  int refinements;         /* F32_REFINE: outer FP64 refinement steps */
  int converged;           /* 1 if every column met rtol */
  int deflations;          /* directions dropped as numerically dependent */
  double max_rel_residual; /* max_j ||r_j|| / ||r0_j|| at exit */
} bkts_solve_info;

/* Solve (alpha I + beta K) X = B for an N x k block with a block Krylov method
 * (block methods: Sec. 1, eq. basic-matrix-equation).  B and X are FP64
 * device blocks; X holds the initial guess on entry and the solution on exit.
 * Convergence is per column; rank deficiency of the block is handled by
 * deflating dependent directions.  Synchronises (reads convergence state). */
bkts_status bkts_block_solve(bkts_ctx ctx, bkts_op op, double alpha, double beta, int k,
                             const double* B, int ldb, double* X, int ldx,
                             const bkts_solve_opts* opts, bkts_solve_info* info);

/* ------------------------------------------------- Algorithm 1 (linear case) */

typedef struct bkts_run_info {
  int accepted_steps;
  int outer_iterations;       /* residual evaluations + block solves (Algorithm 1 inner loop) */
  int krylov_iterations;      /* total block Krylov iterations */
  int refinements;
  double final_front_rel_residual;
} bkts_run_info;

/* Called after each accepted step with the step number (1-based), its time and
 * a DEVICE pointer to y^{n} (N doubles, valid only during the call). */
typedef void (*bkts_step_cb)(int step, double t, const double* y_device, void* user);

/* Algorithm 1 ("Block Krylov Time Stepping with Pipelining") for the linear
 * problem y' + K y = b: a window of k stage columns is iterated with
 * Y <- Y - J^{-1} R(Y), J = I/tau + beta K, until the front column's residual
 * satisfies ||R_0|| <= outer_rtol * ||rhs_0||; the front stage is then
 * accepted and the window shifted (shift(Y_1..Y_k) = (Y_2..Y_k, Y_k)).  For a
 * fully implicit tableau the m columns of the front step must all pass the test
 * and are accepted and shifted out together.  For a DIRK tableau whose implicit
 * diagonal entries differ (a custom tableau), inner->krylov = BKTS_BICGSTAB (a
 * column-wise method) keeps each column's own block J_j = I/tau + A2_jj K: the
 * D (x) M + beta I (x) K form of the remark after eq. matrix-fixed-point-equation,
 * whose splitting is exact after k sweeps; block CG and GMRES use beta = A2_00
 * for every column.
 * `y` (device, N) holds y^0 on entry and y^{n_steps} on exit.  `y_hist`
 * (device, n_steps x N, may be NULL) receives every accepted y^n.  `cb` may
 * be NULL.  Synchronises. */
bkts_status bkts_advance(bkts_ctx ctx, bkts_op op, bkts_tc tc, double* y, int n_steps,
                         const bkts_solve_opts* inner, double outer_rtol, int max_outer,
                         double* y_hist, bkts_step_cb cb, void* user, bkts_run_info* info);

/* One window solved as a whole (linear problem; the outer acceleration the paper names as ongoing
 * work in Sec. 4.1): M Y A1^T + K Y A2^T = b rs^T + B0 with the window matrices of `phase`
 * (Sec. 2.1 eq. general-system-time-steps; rs = row sums of A2), B0 (device, N x nb0, leading
 * dimension ldb0, nb0 <= min(k, 8); NULL = zero) in the first columns.
 *   BKTS_WINDOW_FGMRES:    FGMRES(restart) whose vectors are whole N x k windows (Frobenius inner
 *                          products), right-preconditioned by V -> J^-1 V column by column,
 *                          J = I/tau + beta K, each application one block Krylov solve of the k
 *                          columns with `inner` (eq. matrix-splitting as a preconditioner).
 *   BKTS_WINDOW_SPLITTING: the plain fixed point of eq. matrix-fixed-point-equation,
 *                          Y <- Y + J^-1 (F - L(Y)), for comparison.
 * Y (device, N x k, ld = k) is the initial guess on entry and the solution on exit, to
 * ||R(Y)||_F <= rtol ||F||_F.  At most `maxit` outer iterations; BKTS_ENOCONV (info filled) if the
 * test is not met.  Synchronises. */
enum { BKTS_WINDOW_FGMRES = 0, BKTS_WINDOW_SPLITTING = 1 };
typedef struct bkts_window_info {
  int iterations;            /* outer iterations */
  int inner_iterations;      /* block Krylov iterations of all J^-1 applications */
  int precond_applications;  /* J^-1 applications (block solves of k columns) */
  int converged;
  double rel_residual;       /* ||R(Y)||_F / ||F||_F on return */
} bkts_window_info;
bkts_status bkts_window_solve(bkts_ctx ctx, bkts_op op, bkts_tc tc, int phase, const double* B0, int ldb0, int nb0,
                              double* Y, int method, const bkts_solve_opts* inner, double rtol, int restart,
                              int maxit, bkts_window_info* info);

/* ---------------------------------------------- nonlinear problems (Sec. 2.2) */

/* M y' + f(y) = 0 with f(u) = -div_h(D(u) grad_h u) - r(u) on a cell-centred FV grid,
 * D(u) = sum_i dcoef[i] u^i and r(u) = sum_i rcoef[i] u^i (cubic at most).  Interior faces use
 * the arithmetic mean (D(u_P) + D(u_Q))/2; a Dirichlet face with value g uses (D(u_P) + D(g))/2
 * over half a cell; Neumann faces carry no flux. */
typedef struct bkts_nl_coeffs {
  double dcoef[4];
  double rcoef[4];
  int bc_type[6];      /* face 2*axis + side: BKTS_BC_DIRICHLET or BKTS_BC_NEUMANN */
  double bc_value[6];
} bkts_nl_coeffs;

bkts_status bkts_nlop_create(bkts_ctx ctx, const bkts_grid* grid, const bkts_nl_coeffs* coeffs, bkts_nlop* out);
void bkts_nlop_destroy(bkts_nlop nl);
/* F[:, j] = f(Y[:, j]) for an N x k device block (row-major, leading dimensions ldy, ldf). */
bkts_status bkts_nl_eval(bkts_ctx ctx, bkts_nlop nl, int k, const double* Y, int ldy, double* F, int ldf);
/* Assemble J = alpha m'(u) + beta Df(u) on the stencil sparsity (m' = 1 for the diffusion-reaction
 * operator; see Richards below) (u: device, N doubles) and return it as an operator handle owned
 * by `nl` (valid until the next call or bkts_nlop_destroy; do not destroy it). */
bkts_status bkts_nl_jacobian(bkts_ctx ctx, bkts_nlop nl, const double* u, double alpha, double beta, bkts_op* J);
/* The nonlinear all-at-once residual R = m(Y) A1^T + F(Y) A2^T - B0 (Sec. 2.2; m = identity except
 * for Richards' equation, where m = theta) for the window
 * matrices of `phase`; arguments as bkts_residual. */
bkts_status bkts_nl_residual(bkts_ctx ctx, bkts_nlop nl, bkts_tc tc, int phase, const double* Y, int ldy,
                             const double* B0, int ldb0, int nb0, double* R, int ldr, double* col_norms2);
/* One Newton iteration of Algorithm 1 on the window Y (device N x k, ld = k): R = R(Y);
 * J = I/tau + a_kk Df(Y_0); solve J V = R to opts->rtol per column with the block Krylov method of
 * `opts` (BKTS_PRECISION_F32_REFINE: FP32 inner solves inside FP64 iterative refinement, as
 * bkts_block_solve); Y <- Y - V.
 * col_norms2 (HOST, k, may be NULL) receives ||R_j||^2 of the residual BEFORE the update.
 * Synchronises. */
bkts_status bkts_newton_step(bkts_ctx ctx, bkts_nlop nl, bkts_tc tc, int phase, const double* B0, int ldb0, int nb0,
                             double* Y, double* col_norms2, const bkts_solve_opts* opts, bkts_solve_info* info);

/* Richards' equation (Sec. 4.3): d/dt theta(psi) - div(K(psi) grad(psi + z)) = 0 for the pressure
 * head psi on a cell-centred FV grid of the unit square/cube whose LAST axis is the height z, with
 * the van Genuchten closure of eq. RelationshipsThetaK (theta = theta_r + (theta_s - theta_r) Se,
 * Se = (1 + (alpha |psi|)^n)^(-m), m = 1 - 1/n, Se = 1 for psi >= 0; K = Ks s^(1/2)(1 - (1 -
 * s^(1/m))^m)^2 with s = theta / theta_s as printed in the paper).  Faces: K_f = harmonic mean of
 * Ks times the arithmetic mean of K/Ks; top face Dirichlet psi = top_value (half a cell away) or no
 * flow; bottom face free drainage (unit head gradient, outflow Ks kr(psi)) or no flow; lateral faces
 * no flow.  As an operator for the calls above: f(psi) = -div_h(K grad_h(psi + z)), the mass term
 * is theta(psi) (Algorithm 1 uses theta(Y) A1^T + F(Y) A2^T - B0), and the Jacobian is
 * alpha m'(psi) + beta Df(psi) with m' = theta' (Newton) or the constant lin_L > 0 (L-scheme). */
enum { BKTS_RI_NO_FLOW = 0, BKTS_RI_DIRICHLET = 1, BKTS_RI_FREE_DRAINAGE = 2 };
typedef struct bkts_richards_params {
  double theta_r, theta_s, alpha, n;  /* van Genuchten parameters (n > 1) */
  int top;                            /* BKTS_RI_DIRICHLET or BKTS_RI_NO_FLOW */
  double top_value;                   /* psi on the top face when Dirichlet */
  int bottom;                         /* BKTS_RI_FREE_DRAINAGE or BKTS_RI_NO_FLOW */
  double lin_L;                       /* 0: Newton; > 0: L-scheme constant for theta' */
} bkts_richards_params;
/* ks: device, N saturated conductivities > 0 (copied).  Errors: NULL arguments, dim outside 1..3,
 * n <= 1, alpha <= 0, theta_s <= theta_r < 0, an unknown top/bottom type, lin_L < 0. */
bkts_status bkts_richards_create(bkts_ctx ctx, const bkts_grid* grid, const double* ks,
                                 const bkts_richards_params* params, bkts_nlop* out);
/* M[:, j] = m(Y[:, j]): psi -> theta(psi) for Richards, the identity for the diffusion-reaction
 * operator (device, N x k row-major blocks). */
bkts_status bkts_nl_mass(bkts_ctx ctx, bkts_nlop nl, int k, const double* Y, int ldy, double* M, int ldm);

/* A persistent Algorithm 1 pipeline: the window of k stages and the history
 * of the front step survive between calls, so consecutive
 * bkts_stepper_advance calls continue one time integration (bkts_advance is
 * create + advance + destroy).  y0: device, N doubles, copied at creation. */
typedef struct bkts_stepper_s* bkts_stepper;
bkts_status bkts_stepper_create(bkts_ctx ctx, bkts_op op, bkts_tc tc, const double* y0, bkts_stepper* out);
/* The nonlinear pipeline (Algorithm 1 with Newton: the Jacobian at the front column is rebuilt
 * every outer iteration and used for all columns).  DIRK tableaux only: BKTS_EINVAL for a fully
 * implicit one. */
bkts_status bkts_nl_stepper_create(bkts_ctx ctx, bkts_nlop nl, bkts_tc tc, const double* y0, bkts_stepper* out);
bkts_status bkts_stepper_advance(bkts_stepper st, int n_steps, const bkts_solve_opts* inner, double outer_rtol,
                                 int max_outer, double* y_hist, bkts_step_cb cb, void* user, bkts_run_info* info);
/* Copy the last accepted y^n to the device array y (N doubles; may be NULL) and
 * return the number of steps accepted since creation.  Synchronises. */
bkts_status bkts_stepper_state(bkts_stepper st, double* y, int64_t* accepted);
void bkts_stepper_destroy(bkts_stepper st);


/* ---------------------------------------------------------------- serving */

/* A persistent request loop for ensembles of solves (for example many permeability realisations
 * of one problem).  A worker thread with its own stream admits requests in arrival order as soon
 * as the HBM budget and a slot allow, keeps every admitted solve's state (operator, window, block
 * Krylov vectors and coefficients) resident on the device, and advances all of them together:
 * each round runs one grouped launch per block-CG kernel and block-width class over every solve
 * inside its inner iteration, so requests that arrive while others run share those launches.
 *
 * A request assembles the FV operator of its grid and coefficient field and advances y0 by k
 * implicit stages (for implicit Euler, k time steps), in one of two modes:
 *  - mode 0 (grouped window splitting): the all-at-once system of one window of k stages (Sec.
 *    2.1, eq. general-system-time-steps) by the Newton/splitting iteration (eq.
 *    matrix-fixed-point-equation) until max_j ||R_j|| <= rtol ||rhs_0|| for every column j
 *    (rhs_0 = front column of B A2^T + B0).  Each correction is an FP32 block-CG solve (Jacobi)
 *    of the column-scaled FP64 residual to inner_rtol, grouped with the other mode-0 requests;
 *    residuals and updates are FP64.
 *  - mode 1 (pipelined, implicit Euler only): Algorithm 1 with a window of `window` columns
 *    (0: min(k, 4)), each front column accepted as soon as ||R_0|| <= rtol ||rhs_0|| (Sec. 2.2),
 *    on the index-free stencil form of the operator with FP32 block CG preconditioned by the
 *    geometric multigrid V-cycle (inner_rtol) inside the FP64 outer iteration.  Mode-1 requests
 *    run on min(16, max_slots) worker lanes, each with its own stream, beside the grouped rounds.
 * Both modes share the arrival-order admission and the HBM budget.
 *
 * A request's result does not depend on the other requests in flight: every job keeps its own
 * launch geometry and reduction order. */
typedef struct bkts_server_s* bkts_server;

typedef struct bkts_request {
  bkts_grid grid;
  const double* kappa;   /* device, one value per cell, or NULL for kappa_const */
  double kappa_const;
  int bc_type[6];        /* as bkts_fv_coeffs */
  double bc_value[6];
  const double* y0;      /* device, N values */
  double* y_out;         /* device, N x k row-major: column j = stage j of the window */
  int method;            /* BKTS_IE, BKTS_THETA or BKTS_SDIRK2 */
  double theta;
  int k;                 /* window width, 1..BKTS_MAX_K */
  double tau;
  double rtol;           /* outer tolerance, (0, 1) */
  double inner_rtol;     /* FP32 block-CG per-column relative tolerance, (0, 1) */
  int max_outer;         /* 0: 200 (mode 1: per accepted step) */
  int max_inner;         /* per correction; 0: 2000 */
  uint64_t tag;          /* returned in the result */
  int mode;              /* 0: grouped window splitting; 1: pipelined Algorithm 1 with multigrid */
  int window;            /* mode 1: window width in columns, 0 = min(k, 4) */
} bkts_request;

typedef struct bkts_result {
  uint64_t ticket, tag;
  int status;            /* BKTS_OK, BKTS_ENOCONV, BKTS_EBREAKDOWN, or the setup error */
  int outer_iterations, krylov_iterations;
  double rel_residual;   /* max_j ||R_j|| / ||rhs_0|| at exit (mode 1: the last front column's) */
  double t_submit, t_admit, t_done;  /* seconds on the server clock (bkts_server_clock) */
  size_t footprint_bytes;            /* HBM reserved for the request while it ran */
} bkts_result;

typedef struct bkts_server_stats {
  int queued, active, done_unpolled, max_active;
  long rounds, grouped_launches;
  size_t bytes_in_use, bytes_peak;
} bkts_server_stats;

/* Start a server on ctx's device.  hbm_budget_bytes bounds the sum of the admitted requests'
 * footprints; max_slots (1..256) bounds how many mode-0 requests run at once, and min(16,
 * max_slots) how many mode-1 requests do. */
bkts_status bkts_server_create(bkts_ctx ctx, size_t hbm_budget_bytes, int max_slots, bkts_server* out);
/* Queue a request (non-blocking; thread-safe).  kappa, y0 and y_out must stay valid, and y0 and
 * kappa must already hold their values (the server's stream does not wait for the caller's),
 * until the request's result has been polled.  BKTS_EINVAL for a malformed request; BKTS_ENOMEM
 * if it alone exceeds the budget. */
bkts_status bkts_server_submit(bkts_server srv, const bkts_request* req, uint64_t* ticket);
/* Move up to `max` finished results into out (non-blocking); *n_done = how many.  When a result is
 * returned its y_out is complete.  BKTS_EDEVICE if the worker stopped on a device error. */
bkts_status bkts_server_poll(bkts_server srv, bkts_result* out, int max, int* n_done);
/* Block until at least n results are waiting to be polled or timeout_s passes; *n_ready = count. */
bkts_status bkts_server_wait(bkts_server srv, int n, double timeout_s, int* n_ready);
bkts_status bkts_server_stats_get(bkts_server srv, bkts_server_stats* out);
/* Seconds since the server was created (the clock of bkts_result). */
double bkts_server_clock(bkts_server srv);
/* Finish the admitted requests, drop the queued ones, stop the worker and free everything. */
void bkts_server_destroy(bkts_server srv);

#ifdef __cplusplus
}
#endif
#endif /* BKTS_H */

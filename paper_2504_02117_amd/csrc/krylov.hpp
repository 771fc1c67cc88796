// Block Krylov solvers (krylov.cpp).
#pragma once

#include <functional>

#include "internal.hpp"

namespace bkts {

// A different operator per column: column j of the block solves (a[j] I + b[j] K) x_j = r_j.  This
// is the left-hand side D (x) M + beta I (x) K of the remark after eq. matrix-fixed-point-equation
// (M the identity, D diagonal), after each column is divided by its own beta: the columns' Krylov
// spaces are those of K, so the column-wise (vectorized) methods solve every column with its own
// shift.  Entries in the physical column order of the block.
struct ColOp {
  double a[BKTS_MAX_K];
  double b[BKTS_MAX_K];
};

struct KrylovStats {
  int iterations = 0;
  int refinements = 0;
  int converged = 0;
  int deflations = 0;
  int breakdown = 0;  // the method stopped early on a breakdown and returned its last iterate
  double max_rel = 0.0;
};

// Block CG for (a I + b K) X = B on contiguous blocks of type dtype.  X is the initial guess
// (ignored and treated as zero when x0_zero).  Per-column relative tolerance rtol.
void block_cg(bkts_ctx ctx, const bkts_op_s& op, int dtype, int k, double a, double b, const void* B, void* X,
              bool x0_zero, bool jacobi, double rtol, int maxit, KrylovStats& st);

void block_gmres(bkts_ctx ctx, const bkts_op_s& op, int dtype, int k, double a, double b, const void* B, void* X,
                 bool x0_zero, bool jacobi, double rtol, int restart, int maxit, KrylovStats& st,
                 const bkts_op_s* mgop = nullptr);

// Block GMRES(m) on an operator given by callbacks, on contiguous N x k blocks of type dtype:
// apply: out = A in; precond: out = P in (right preconditioner); residual: W = B - A X (when
// x0_zero, also set X = 0).  flexible keeps P V_j for every j (FGMRES).  Workspace names start
// with ws_prefix, so a preconditioner may itself run block GMRES under another prefix.
struct GmresOps {
  std::function<void(const void*, void*)> apply;
  std::function<void(const void*, void*)> precond;
  std::function<void(const void*, void*, bool, void*)> residual;
  bool flexible = false;
  const char* ws_prefix = "gm";
};
void gmres_core(bkts_ctx ctx, int dtype, int64_t N, int k, const GmresOps& ops, const void* B, void* X,
                bool x0_zero, double rtol, int restart, int maxit, KrylovStats& st);
// cop != nullptr: column j's operator is cop->a[j] I + cop->b[j] K (the Jacobi scaling stays that
// of a I + b K).  mgop != nullptr: right-preconditioned by one multigrid V-cycle for a I + b K_mg,
// with K_mg the stencil form of mgop (the operator itself, or the symmetric part of a Jacobian).
void block_bicgstab(bkts_ctx ctx, const bkts_op_s& op, int dtype, int k, double a, double b, const void* B, void* X,
                    bool x0_zero, bool jacobi, double rtol, int maxit, KrylovStats& st, const ColOp* cop = nullptr,
                    const bkts_op_s* mgop = nullptr);

// What a caller already knows about a solve's right-hand side: its squared column norms (host; only
// with a zero initial guess), and that it is scratch the solver may overwrite.
struct SolveHints {
  const double* nrm0 = nullptr;
  bool b_scratch = false;
};

// One FP32 correction inside a caller's FP64 outer loop: Y += coef * (a M + b K)^-1 R, where the
// caller's residual kernel already produced R's squared column norms (on the device and the host).
// R is scaled to unit columns in FP32, solved to the options' inner tolerance, and the correction is
// scaled back and accumulated into Y in the same pass (no FP64 correction block).
void correct_f32(bkts_ctx ctx, const bkts_op_s& op, double a, double b, int k, const double* R, const double* rn2_dev,
                 const double* rn2_host, double coef, double* Y, const bkts_solve_opts& o, KrylovStats& st,
                 const ColOp* cop = nullptr);

// FP64 solve entry: F64 block CG, or FP32 block CG inside FP64 iterative refinement.  With
// single_f32_pass the refinement loop makes one FP32 correction (the caller's own outer loop
// computes FP64 residuals).
// With cop (vectorized BiCGStab only, one FP32 pass or FP64): the per-column operators of ColOp;
// (a, b) then only set the Jacobi scaling.
void solve(bkts_ctx ctx, const bkts_op_s& op, double a, double b, int k, const double* B, double* X, bool x0_zero,
           const bkts_solve_opts& o, bool single_f32_pass, KrylovStats& st, const ColOp* cop = nullptr);

}  // namespace bkts

// Krylov-accelerated solve of one all-at-once window (accel.cpp).
#pragma once

#include "internal.hpp"

namespace bkts {

struct WindowStats {
  int iterations = 0;            // outer (FGMRES or splitting) iterations
  int inner_iterations = 0;      // block Krylov iterations over all preconditioner applications
  int precond_applications = 0;  // block solves with J
  int converged = 0;
  double rel_residual = 0.0;     // ||R(Y)||_F / ||F||_F at return
};

// Solve M Y A1^T + K Y A2^T = b rs^T + B0 for the window of `phase` (logical = physical columns)
// from the initial guess Y (N x k, ld k), by FGMRES(restart) with the J^-1 block solve as right
// preconditioner (BKTS_WINDOW_FGMRES) or by the plain splitting iteration (BKTS_WINDOW_SPLITTING),
// to ||R||_F <= rtol ||F||_F.
void window_solve(bkts_ctx ctx, const bkts_op_s& op, const bkts_tc_s& tc, int phase, const double* B0, int ldb0,
                  int nb0, double* Y, const bkts_solve_opts& inner, int method, double rtol, int restart, int maxit,
                  WindowStats& out);

}  // namespace bkts

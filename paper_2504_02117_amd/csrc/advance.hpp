// Algorithm 1, linear and Newton forms (advance.cpp).
#pragma once

#include <vector>

#include "internal.hpp"

// Persistent pipeline state of Algorithm 1: the window and the history of the front step.
struct bkts_stepper_s {
  bkts_ctx ctx;
  bkts_op op;          // linear operator K, or the Jacobian storage of `nl`
  bkts_tc tc;
  bkts_nlop nl = nullptr;  // nonlinear problem (Newton form) or null
  bkts::DevBuf Y, R, V, B0, fst, yprev, fyn, tmp, nrm;
  bkts::DevBuf mats;  // window matrices (A1, A2, row sums of A2) of every (phase, off), in that order
  int off = 0;       // physical column of logical column 0
  // implicit Euler windows (A1 = (I - L)/tau, A2 = I, one stage): a shift leaves the residual of
  // every kept column unchanged, and the duplicated last column's residual is K y - b
  bool ie_window = false;
  int phase = 0;     // implicit-stage index of the front column within its step
  long accepted = 0; // accepted steps since creation
  bkts_stepper_s(bkts_ctx c, bkts_op o, bkts_tc t, const double* y0, bkts_nlop n = nullptr);
  void eval_f(const double* x, int ldx, double* out, int ldo);
  bkts_status advance(int n_steps, const bkts_solve_opts& inner, double outer_rtol, int max_outer, double* y_hist,
                      bkts_step_cb cb, void* user, bkts_run_info* info);
  void guard_window(int it, int off, const std::vector<double>& hn, std::vector<double>& ref,
                    std::vector<char>& active, std::vector<char>& frozen);
};

namespace bkts {

void window_mats(const bkts_tc_s& tc, int phase, int off, double* h);
void upload_window(bkts_ctx ctx, const bkts_tc_s& tc, int phase, int off, double* A1p, double* A2p, double* rsp);

// Residual of the window whose logical column 0 is physical column `off` (ring layout).  `mats`
// holds the uploaded physical window matrices, or is null to upload them here.
void window_residual(bkts_ctx ctx, const bkts_op_s& op, const bkts_tc_s& tc, int phase, int off, const double* Y,
                     int ldy, const double* B0, int ldb0, int nb0, double* R, int ldr, double* nrm_dev,
                     double* mats = nullptr);

bkts_status advance(bkts_ctx ctx, bkts_op op, bkts_tc tc, double* y, int n_steps, const bkts_solve_opts& inner,
                    double outer_rtol, int max_outer, double* y_hist, bkts_step_cb cb, void* user,
                    bkts_run_info* info);

}  // namespace bkts

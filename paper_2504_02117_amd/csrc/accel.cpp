// Outer acceleration of one window of Algorithm 1, linear case.  The paper loosens the inner
// tolerance so that extra outer iterations refresh the right-hand sides of the later columns, and
// names updating those right-hand sides inside the Krylov solver itself as ongoing work (Sec. 4.1).
// Here the whole window is the unknown of one Krylov method: FGMRES(m) on the all-at-once operator
// L(Y) = M Y A1^T + K Y A2^T (Sec. 2.1, eq. general-system-time-steps; a vector is the N x k window,
// inner products are Frobenius), right-preconditioned by the splitting's approximate inverse
// P(V) = J^-1 V, J = M/tau + beta K (eq. matrix-splitting), column by column.  Each application of
// P is one block Krylov solve of all k columns, so the flexible variant keeps every P V_j.  The
// plain splitting iteration of eq. matrix-fixed-point-equation, Y <- Y + P(F - L Y), is the same
// loop without the Krylov acceleration and is kept for comparison.
#include <cmath>

#include "accel.hpp"
#include "advance.hpp"
#include "krylov.hpp"
#include "vecops.hpp"

namespace bkts {

void window_solve(bkts_ctx ctx, const bkts_op_s& op, const bkts_tc_s& tc, int phase, const double* B0, int ldb0,
                  int nb0, double* Y, const bkts_solve_opts& inner, int method, double rtol, int restart, int maxit,
                  WindowStats& out) {
  const int64_t N = op.N;
  const int k = tc.k;
  const int64_t n = N * k;
  const double tau = tc.tau;
  const double beta = tc_beta(tc, phase);
  const size_t nm = 2 * (size_t)k * k + k;
  double* mats = ctx->ws.get<double>("acc_mats", 2 * nm);  // window matrices, then a copy with zero row sums
  double* matsL = mats + nm;
  upload_window(ctx, tc, phase, 0, mats, nullptr, nullptr);
  BKTS_HIP(hipMemcpyAsync(matsL, mats, sizeof(double) * 2 * k * k, hipMemcpyDeviceToDevice, ctx->stream));
  BKTS_HIP(hipMemsetAsync(matsL + 2 * k * k, 0, sizeof(double) * k, ctx->stream));
  double* nrm = ctx->ws.get<double>("acc_nrm", k);
  double* W0 = ctx->ws.get<double>("acc_w0", n);
  double* Z = ctx->ws.get<double>("acc_z", n);  // zero input for ||F||, then the splitting's correction
  int cols[8];
  for (int i = 0; i < 8; ++i) cols[i] = i;
  const int nb = B0 ? nb0 : 0;
  auto fro2 = [&]() {  // sum of the k column norms^2 of the last residual launch
    double* hs = ctx->host_stage(k);
    BKTS_HIP(hipMemcpyAsync(hs, nrm, sizeof(double) * k, hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += hs[j];
    return s;
  };
  // W = F - L(X) = -R(X), with F = b rs^T + B0 the window's right-hand side
  auto neg_residual = [&](const double* X, double* W) {
    residual(ctx, op, k, X, k, mats, mats + k * k, mats + 2 * k * k, B0, ldb0, nb, cols, W, k, nrm);
    axpby(ctx, n, 0.0, W, -1.0, W);
  };
  auto precond = [&](const double* V, double* PV) {
    KrylovStats s;
    solve(ctx, op, 1.0 / tau, beta, k, V, PV, true, inner, true, s);
    out.inner_iterations += s.iterations;
    ++out.precond_applications;
  };
  out = WindowStats{};
  // ||F|| from the residual at zero (input and output must not alias: the stencil reads neighbours)
  BKTS_HIP(hipMemsetAsync(Z, 0, sizeof(double) * n, ctx->stream));
  residual(ctx, op, k, Z, k, mats, mats + k * k, mats + 2 * k * k, B0, ldb0, nb, cols, W0, k, nrm);
  const double fnorm = std::sqrt(fro2());
  if (!(fnorm > 0.0)) {  // zero right-hand side: the solution is zero
    BKTS_HIP(hipMemsetAsync(Y, 0, sizeof(double) * n, ctx->stream));
    ctx->sync();
    out.converged = 1;
    return;
  }
  neg_residual(Y, W0);
  double r = std::sqrt(fro2());
  if (!std::isfinite(r)) throw Error{BKTS_EBREAKDOWN, "non-finite window residual"};
  if (method == BKTS_WINDOW_SPLITTING) {
    while (r > rtol * fnorm && out.iterations < maxit) {
      precond(W0, Z);
      axpby(ctx, n, 1.0, Z, 1.0, Y);
      neg_residual(Y, W0);
      r = std::sqrt(fro2());
      if (!std::isfinite(r)) throw Error{BKTS_EBREAKDOWN, "non-finite window residual"};
      ++out.iterations;
    }
  } else if (r > rtol * fnorm) {
    GmresOps ops;
    ops.ws_prefix = "wg";
    ops.flexible = true;
    ops.apply = [&](const void* in, void* o) {  // L(Z): the residual kernel without b and B0 terms
      residual(ctx, op, k, static_cast<const double*>(in), k, matsL, matsL + k * k, matsL + 2 * k * k, nullptr, 0,
               0, cols, static_cast<double*>(o), k, nrm);
    };
    ops.precond = [&](const void* in, void* o) { precond(static_cast<const double*>(in), static_cast<double*>(o)); };
    ops.residual = [&](const void*, void* X, bool, void* W) {
      neg_residual(static_cast<const double*>(X), static_cast<double*>(W));
    };
    KrylovStats st;
    // relative to the initial residual inside the core; rescaled so the test is ||R|| <= rtol ||F||
    gmres_core(ctx, BKTS_F64, n, 1, ops, nullptr, Y, false, rtol * fnorm / r, restart, maxit, st);
    out.iterations = st.iterations;
    neg_residual(Y, W0);
    r = std::sqrt(fro2());
  }
  out.rel_residual = r / fnorm;
  out.converged = r <= rtol * fnorm ? 1 : 0;
}

}  // namespace bkts

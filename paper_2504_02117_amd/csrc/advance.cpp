#include <algorithm>
// Algorithm 1 (Block Krylov Time Stepping with Pipelining) for the linear problem y' + K y = b.
//
// The window Y holds k consecutive implicit stages.  Each outer iteration forms the fused FP64
// residual R(Y) = Y A1^T + (K Y - b 1^T) A2^T - B0, tests the front column, and applies the
// Newton/splitting update Y <- Y - J^{-1} R with J = I/tau + beta K (in the linear case this
// update is exactly one sweep of eq. matrix-fixed-point-equation).  When the front stage has
// converged it is accepted and the window is shifted, shift(Y_1..Y_k) = (Y_2..Y_k, Y_k).
//
// The window is a ring buffer: logical column i lives in physical column (off + i) mod k, so a
// shift costs one column copy instead of moving the whole block; the k x k couplings and the B0
// columns are permuted to the physical order instead.  A stepper keeps the window between calls,
// so consecutive advance calls continue one pipeline.
#include <cmath>
#include <cstring>

#include "advance.hpp"
#include "krylov.hpp"
#include "vecops.hpp"

namespace bkts {

// The window matrices of (phase, off) in physical column order: A1, A2 and the row sums of A2.
void window_mats(const bkts_tc_s& tc, int phase, int off, double* h) {
  const int k = tc.k;
  for (int i = 0; i < k; ++i) {
    const int pi = (off + i) % k;
    double rs = 0.0;
    for (int j = 0; j < k; ++j) {
      const int pj = (off + j) % k;
      h[pi * k + pj] = tc.A1[phase][i * k + j];
      h[k * k + pi * k + pj] = tc.A2[phase][i * k + j];
      rs += tc.A2[phase][i * k + j];
    }
    h[2 * k * k + pi] = rs;
  }
}

void upload_window(bkts_ctx ctx, const bkts_tc_s& tc, int phase, int off, double* A1p, double* A2p, double* rsp) {
  const int k = tc.k;
  double* h = ctx->host_stage(2 * k * k + k);
  ctx->sync();  // the staging buffer may still be the target of an earlier read-back
  window_mats(tc, phase, off, h);
  BKTS_HIP(hipMemcpyAsync(A1p, h, sizeof(double) * (2 * k * k + k), hipMemcpyHostToDevice, ctx->stream));
  (void)A2p;
  (void)rsp;
  ctx->sync();
}

void window_residual(bkts_ctx ctx, const bkts_op_s& op, const bkts_tc_s& tc, int phase, int off, const double* Y,
                     int ldy, const double* B0, int ldb0, int nb0, double* R, int ldr, double* nrm_dev,
                     double* mats) {
  const int k = tc.k;
  if (!mats) {
    mats = ctx->ws.get<double>("win_mats", 2 * k * k + k);
    upload_window(ctx, tc, phase, off, mats, mats + k * k, mats + 2 * k * k);
  }
  int cols[8];
  for (int i = 0; i < nb0 && i < 8; ++i) cols[i] = (off + i) % k;
  residual(ctx, op, k, Y, ldy, mats, mats + k * k, mats + 2 * k * k, B0, ldb0, nb0, cols, R, ldr, nrm_dev);
}

static void read_vec(bkts_ctx ctx, const double* dev, int n, std::vector<double>& out) {
  double* h = ctx->host_stage(n);
  BKTS_HIP(hipMemcpyAsync(h, dev, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
  ctx->sync();
  out.assign(h, h + n);
}

}  // namespace bkts

bkts_stepper_s::bkts_stepper_s(bkts_ctx c, bkts_op o, bkts_tc t, const double* y0, bkts_nlop n)
    : ctx(c), op(o), tc(t), nl(n) {
  using namespace bkts;
  const int64_t N = op->N;
  const int k = tc->k;
  const int mi = tc->m_impl;
  Y.alloc(sizeof(double) * N * k);
  R.alloc(sizeof(double) * N * k);
  V.alloc(sizeof(double) * N * k);
  B0.alloc(sizeof(double) * N * mi);
  fst.alloc(sizeof(double) * N * mi);
  yprev.alloc(sizeof(double) * N);
  fyn.alloc(sizeof(double) * N);
  tmp.alloc(sizeof(double) * N);
  nrm.alloc(sizeof(double) * (k + 1));
  // the window matrices of every (phase, off), uploaded once: the window shifts without a host
  // round trip
  {
    const size_t per = (size_t)(2 * k * k + k);
    std::vector<double> h(per * mi * k);
    for (int ph = 0; ph < mi; ++ph)
      for (int o = 0; o < k; ++o) window_mats(*tc, ph, o, h.data() + per * (ph * k + o));
    mats.alloc(sizeof(double) * h.size());
    BKTS_HIP(hipMemcpyAsync(mats.p, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, ctx->stream));
    ctx->sync();  // h is pageable and goes out of scope
  }
  if (mi == 1 && !tc->fully_implicit && !tc->explicit_first && k >= 2) {
    const double it = 1.0 / tc->tau;
    bool ie = true;
    for (int i = 0; i < k && ie; ++i)
      for (int j = 0; j < k && ie; ++j) {
        const double a1 = i == j ? it : (j == i - 1 ? -it : 0.0), a2 = i == j ? 1.0 : 0.0;
        ie = std::fabs(tc->A1[0][i * k + j] - a1) <= 1e-14 * it && tc->A2[0][i * k + j] == a2;
      }
    ie_window = ie;
  }
  // Algorithm 1 starts from Y = (y0, ..., y0)
  broadcast_cols(ctx, N, k, y0, Y.as<double>(), k);
  BKTS_HIP(hipMemcpyAsync(yprev.p, y0, sizeof(double) * N, hipMemcpyDeviceToDevice, ctx->stream));
  if (tc->explicit_first) eval_f(yprev.as<double>(), 1, fyn.as<double>(), 1);
  ctx->sync();
}

void bkts_stepper_s::eval_f(const double* x, int ldx, double* out, int ldo) {  // f(x) = K x - b, or nonlinear f
  if (nl) return bkts::nl_eval(ctx, *nl, 1, x, ldx, out, ldo);
  const double* bsrc = op->b_nonzero ? op->b.as<double>() : nullptr;
  bkts::spmm(ctx, *op, BKTS_F64, 1, -1.0, bsrc, 1, 0.0, x, ldx, 1.0, out, ldo);
}

// Safeguard of the Newton form (not part of Algorithm 1): the later slots of the window are
// updated with the front stage's Jacobian, and when the problem changes quickly over the window
// (a wetting front in Richards' equation) their iterates can diverge even though the front stage
// converges.  A later slot whose residual norm becomes non-finite or exceeds kGrowth times its norm
// at stage entry is rolled back by its last update and takes no further update this stage; at the
// shift it restarts from the converged front stage, the initial guess sequential stepping would
// use.  The front stage is never touched, so the accepted steps are those of plain Newton.
void bkts_stepper_s::guard_window(int it, int off, const std::vector<double>& hn, std::vector<double>& ref,
                                  std::vector<char>& active, std::vector<char>& frozen) {
  using namespace bkts;
  constexpr double kGrowth = 10.0;
  const int64_t N = op->N;
  const int k = tc->k;
  double* Yp = Y.as<double>();
  double* Rp = R.as<double>();
  double* Vp = V.as<double>();
  for (int j = 0; j < k; ++j) {
    if (j == off) continue;
    const double r = std::sqrt(hn[j]);
    if (it == 0) {
      ref[j] = r;
      if (std::isfinite(r)) continue;
      copy_col(ctx, N, Yp, k, off, j);  // defensive: no finite iterate to roll back to
    } else {
      if (!active[j] || (std::isfinite(r) && r <= kGrowth * ref[j])) continue;
      LinComb back;  // Y_j += V_j undoes the last update
      back.add(1.0, Yp + j, k);
      back.add(1.0, Vp + j, k);
      lincomb(ctx, N, back, Yp + j, k);
    }
    active[j] = 0;
    frozen[j] = 1;
    copy_col(ctx, N, Rp, k, off, j);  // a finite right-hand side for the block solve
  }
}

bkts_status bkts_stepper_s::advance(int n_steps, const bkts_solve_opts& inner, double outer_rtol, int max_outer,
                                    double* y_hist, bkts_step_cb cb, void* user, bkts_run_info* info) {
  using namespace bkts;
  const int64_t N = op->N;
  const int k = tc->k;
  const int mi = tc->m_impl;
  const double tau = tc->tau;
  const double* bsrc = (!nl && op->b_nonzero) ? op->b.as<double>() : nullptr;
  double* Yp = Y.as<double>();
  double* Rp = R.as<double>();
  double* Vp = V.as<double>();
  double* B0p = B0.as<double>();
  double* fstp = fst.as<double>();
  double* yp = yprev.as<double>();
  double* nrmp = nrm.as<double>();
  bkts_run_info ri{};
  std::vector<double> hn;
  // Newton form: per window slot, the residual norm at stage entry, whether the slot still takes
  // updates this stage, and whether it was frozen this stage.
  std::vector<double> ref(k, 0.0);
  std::vector<char> active(k, 1), frozen(k, 0);
  bkts_status status = BKTS_OK;
  int done = 0;
  bool shifted = false;  // the window was shifted after a full residual of the unshifted window
  while (done < n_steps) {
    // B0 columns of the window: stages q = phase + i of the front step (Sec. 2.2)
    const int nb0 = std::min(mi - phase, k);
    // m(y^n): identity, or theta(psi^n) for Richards' equation
    const double* myp = yp;
    if (nl && nl->nd.kind != 0) {
      nl_mass(ctx, *nl, 1, yp, 1, tmp.as<double>(), 1);
      myp = tmp.as<double>();
    }
    for (int i = 0; i < nb0; ++i) {
      const int q = phase + i;
      LinComb lc;
      lc.add(1.0 / tau, myp, 1);
      for (int j = 0; j < phase; ++j) lc.add(-tc->Ai[q * mi + j], fstp + j, mi);
      if (tc->explicit_first) lc.add(-tc->ae[q], fyn.as<double>(), 1);
      lincomb(ctx, N, lc, B0p + i, mi);
    }
    // scale of the front equation: ||(B A2^T)_0 + B0_0||
    {
      LinComb lc;
      double rs0 = 0.0;
      for (int j = 0; j < k; ++j) rs0 += tc->A2[phase][j];
      if (bsrc) lc.add(rs0, bsrc, 1);
      lc.add(1.0, B0p, mi);
      lincomb(ctx, N, lc, tmp.as<double>(), 1);
      colnorms2(ctx, BKTS_F64, N, 1, tmp.as<double>(), 1, nrmp + k);
    }
    double* matsp = mats.as<double>() + (size_t)(2 * k * k + k) * (phase * k + off);
    const double beta = tc_beta(*tc, phase);
    // A DIRK window whose diagonal coefficients differ (a custom tableau with distinct a_ii): with a
    // column-wise inner method, each column keeps its own diagonal block M/tau + A2_jj K, the
    // D (x) M + beta I (x) K form of the remark after eq. matrix-fixed-point-equation, instead of
    // moving (A2_jj - beta) K to the right-hand side.
    ColOp cop;
    bool col_ops = false;
    if (!nl && !tc->fully_implicit && inner.krylov == BKTS_BICGSTAB) {
      for (int i = 0; i < k; ++i) {
        const int p = (off + i) % k;  // physical column of window slot i
        cop.a[p] = tc->A1[phase][i * k + i];
        cop.b[p] = tc->A2[phase][i * k + i];
        col_ops = col_ops || cop.b[p] != beta || cop.a[p] != 1.0 / tau;
      }
    }
    // columns accepted together: the front stage, or every stage of the front step when the
    // tableau is fully implicit (its first stage couples to the later ones of the same step)
    const int nacc = tc->fully_implicit ? mi : 1;
    bool front_ok = false;
    for (int it = 0;; ++it) {
      if (nl) {
        int cols[8];
        for (int i = 0; i < nb0 && i < 8; ++i) cols[i] = (off + i) % k;
        double* m = matsp;
        nl_residual(ctx, *nl, k, Yp, k, m, m + k * k, B0p, mi, nb0, cols, Rp, k, nrmp);
      } else if (it == 0 && shifted && ie_window) {
        // after an implicit-Euler shift the kept columns, the new front included (its B0 term is the
        // accepted column it was coupled to), keep their residuals and norms; only the duplicated
        // last column, whose time difference is zero, needs R = K y - b
        const int c = (off + k - 1) % k;
        spmm(ctx, *op, BKTS_F64, 1, -1.0, bsrc, 1, 0.0, Yp + c, k, 1.0, Rp + c, k);
        colnorms2(ctx, BKTS_F64, N, 1, Rp + c, k, nrmp + c);
      } else {
        window_residual(ctx, *op, *tc, phase, off, Yp, k, B0p, mi, nb0, Rp, k, nrmp, matsp);
      }
      read_vec(ctx, nrmp, k + 1, hn);
      const double rhs0 = std::sqrt(hn[k]);
      double front2 = 0.0;
      for (int i = 0; i < nacc; ++i) front2 = std::max(front2, hn[(off + i) % k]);
      const double front = std::sqrt(front2);
      if (nl && k > 1) guard_window(it, off, hn, ref, active, frozen);
      ri.final_front_rel_residual = rhs0 > 0.0 ? front / rhs0 : front;
      if (!std::isfinite(front)) throw Error{BKTS_EBREAKDOWN, "non-finite residual in the time window"};
      if (front <= outer_rtol * rhs0) {
        front_ok = true;
        break;
      }
      if (it >= max_outer) break;
      KrylovStats ks;
      if (nl) {  // Newton: J = I/tau + a_kk Df(front column), used for every column of the window
        nl_jacobian(ctx, *nl, Yp + off, k, 1.0 / tau, beta);
        solve(ctx, *nl->jac, 0.0, 1.0, k, Rp, Vp, true, inner, true, ks);
        for (int j = 0; j < k; ++j)
          if (!active[j]) lincomb(ctx, N, LinComb{}, Vp + j, k);  // frozen slots take no update
      } else if (inner.precision == BKTS_PRECISION_F32_REFINE) {
        // Y <- Y - J^-1 R in one FP32 pass, scaled by the residual kernel's column norms
        correct_f32(ctx, *op, 1.0 / tau, beta, k, Rp, nrmp, hn.data(), -1.0, Yp, inner, ks, col_ops ? &cop : nullptr);
      } else {
        solve(ctx, *op, 1.0 / tau, beta, k, Rp, Vp, true, inner, true, ks, col_ops ? &cop : nullptr);
      }
      ri.krylov_iterations += ks.iterations;
      ri.refinements += ks.refinements;
      ++ri.outer_iterations;
      if (nl || inner.precision != BKTS_PRECISION_F32_REFINE) axpby(ctx, N * k, -1.0, Vp, 1.0, Yp);  // Y <- Y - V
    }
    if (!front_ok) {
      status = BKTS_ENOCONV;
      set_last_error(fmt("front stage not converged after %d outer iterations (rel. residual %.3e)", max_outer,
                         ri.final_front_rel_residual));
      break;
    }
    // slots frozen during this stage restart from the converged front stage
    if (nl) {
      for (int j = 0; j < k; ++j)
        if (frozen[j] && j != off) copy_col(ctx, N, Yp, k, off, j);
      std::fill(frozen.begin(), frozen.end(), 0);
      std::fill(active.begin(), active.end(), 1);
    }
    // accept the front stage (the whole front step for a fully implicit tableau)
    bool shifted_now = false;  // the front slot already holds the duplicated last column
    if (tc->fully_implicit || phase == mi - 1) {
      if (nacc == 1) {  // take the front column and duplicate the last into its slot, in one pass
        take_and_replace_col(ctx, N, Yp, k, off, (off + k - 1) % k, yp);
        shifted_now = true;
      } else {
        extract_col(ctx, N, Yp, k, (off + nacc - 1) % k, yp);
      }
      ++done;
      ++accepted;
      if (y_hist)
        BKTS_HIP(hipMemcpyAsync(y_hist + (size_t)(done - 1) * N, yp, sizeof(double) * N, hipMemcpyDeviceToDevice,
                                ctx->stream));
      if (cb) {
        ctx->sync();
        cb(accepted, accepted * tau, yp, user);
      }
      if (tc->explicit_first) eval_f(yp, 1, fyn.as<double>(), 1);
      phase = 0;
    } else {
      eval_f(Yp + off, k, fstp + phase, mi);
      ++phase;
    }
    for (int i = 0; i < nacc; ++i) {  // shift: duplicate the last column
      if (!shifted_now) copy_col(ctx, N, Yp, k, (off + k - 1) % k, off);
      off = (off + 1) % k;
    }
    shifted = true;
  }
  ctx->sync();
  ri.accepted_steps = done;
  if (info) *info = ri;
  return status;
}

namespace bkts {

bkts_status advance(bkts_ctx ctx, bkts_op op, bkts_tc tc, double* y, int n_steps, const bkts_solve_opts& inner,
                    double outer_rtol, int max_outer, double* y_hist, bkts_step_cb cb, void* user,
                    bkts_run_info* info) {
  bkts_stepper_s st(ctx, op, tc, y);
  bkts_status s = st.advance(n_steps, inner, outer_rtol, max_outer, y_hist, cb, user, info);
  BKTS_HIP(hipMemcpyAsync(y, st.yprev.p, sizeof(double) * op->N, hipMemcpyDeviceToDevice, ctx->stream));
  ctx->sync();
  return s;
}

}  // namespace bkts

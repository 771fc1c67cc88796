// Block GMRES(m) and block BiCGStab for nonsymmetric (a I + b K) X = B (convection, Newton
// Jacobians), right-preconditioned with Jacobi: A D^-1 U = B, X = D^-1 U.  All coefficient
// matrices (block Hessenberg, CholQR factors, k x k systems) stay on the device in FP64; the host
// reads only the k residual norms per iteration.
//
// Block GMRES: block Arnoldi with classical block Gram-Schmidt applied twice and CholQR2 for the
// new block (directions that CholQR finds dependent are dropped), then the small least-squares
// problem min || [S;0] - Hbar Y || by Householder reflectors updated one block column per iteration
// on one workgroup.  The core takes the operator, the right preconditioner and the residual as
// callbacks; with `flexible` it keeps every preconditioned direction (FGMRES), for preconditioners
// that change from one application to the next (an inner Krylov solve).
// Block BiCGStab (Guennouni-Jbilou-Sadok form): k x k alpha and beta from the shadow Gram
// Rt^T V, a scalar omega = <T,S>_F / <T,T>_F.
#include <algorithm>
#include <cmath>

#include "krylov.hpp"
#include "vecops.hpp"

namespace bkts {

namespace {

void read_host(bkts_ctx ctx, const double* dev, int n, std::vector<double>& out) {
  double* h = ctx->host_stage(n);
  BKTS_HIP(hipMemcpyAsync(h, dev, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
  ctx->sync();
  out.assign(h, h + n);
}

bool converged(const std::vector<double>& nrm2, const std::vector<double>& nrm0, double rtol, double* maxrel,
               bool squared) {
  bool ok = true;
  double mr = 0.0;
  for (size_t j = 0; j < nrm2.size(); ++j) {
    const double r = squared ? std::sqrt(nrm2[j]) : nrm2[j];
    const double r0 = std::sqrt(nrm0[j]);
    if (!std::isfinite(r)) throw Error{BKTS_EBREAKDOWN, fmt("non-finite residual in column %zu", j)};
    const double rel = r0 > 0.0 ? r / r0 : (r > 0.0 ? INFINITY : 0.0);
    mr = std::max(mr, rel);
    if (!(r <= rtol * r0)) ok = false;
  }
  if (maxrel) *maxrel = mr;
  return ok;
}

}  // namespace

void gmres_core(bkts_ctx ctx, int dtype, int64_t N, int k, const GmresOps& ops, const void* B, void* X,
                bool x0_zero, double rtol, int restart, int maxit, KrylovStats& st) {
  const size_t es = esize(dtype);
  const size_t blk = es * N * k;
  BKTS_REQUIRE(gmres_max_rows(k) / k >= 2, "block GMRES: block width %d too large", k);
  const int m = std::max(1, std::min(restart > 0 ? restart : 30, gmres_max_rows(k) / k - 1));
  const std::string pre = std::string(ops.ws_prefix) + (dtype == BKTS_F64 ? "_d" : "_s");
  char* V = static_cast<char*>(ctx->ws.get(pre + "_V", blk * (m + 1)));
  char* Zs = ops.flexible ? static_cast<char*>(ctx->ws.get(pre + "_Zs", blk * m)) : nullptr;
  void* W = ctx->ws.get(pre + "_W", blk);
  void* Z = ctx->ws.get(pre + "_Z", blk);
  const int ldh = (m + 1) * k;
  const size_t kk = (size_t)k * k;
  const size_t hsz = (size_t)ldh * m * k;
  double* sm = ctx->ws.get<double>(pre + "_small", 2 * hsz + (size_t)m * k * (2 * k + 1) + (size_t)ldh * k + 8 * kk +
                                                       (size_t)m * k * k + 4 * k + 2);
  double* H = sm;
  double* Rq = H + hsz;                   // triangular factor of H
  double* Vr = Rq + hsz;                  // Householder vectors, 2k per column
  double* Br = Vr + (size_t)m * k * 2 * k;
  double* Gq = Br + (size_t)m * k;        // Q^T [S; 0]
  double* S = Gq + (size_t)ldh * k;
  double* Gm = S + kk;
  double* Ri1 = Gm + kk;
  double* R1 = Ri1 + kk;
  double* Ri2 = R1 + kk;
  double* R2 = Ri2 + kk;
  double* Hb = R2 + kk;
  double* Tm = Hb + kk;
  double* Y = Tm + kk;
  double* resn = Y + (size_t)m * k * k;
  double* nrmd = resn + k;
  const double eps = dtype == BKTS_F64 ? 1e-13 : 1e-6;
  const double lsq_eps = dtype == BKTS_F64 ? 1e-14 : 1e-7;
  auto Vb = [&](int j) { return static_cast<void*>(V + blk * j); };
  auto Zb = [&](int j) { return ops.flexible ? static_cast<void*>(Zs + blk * j) : Z; };
  // CholQR2 of the block `src` into `dst` (may alias): dst R = src, R = R2 R1 stored in Rout.
  auto cholqr2 = [&](void* src, void* dst, double* Rout) {
    gram(ctx, dtype, N, k, src, k, src, k, Gm);
    small_cholqr(ctx, k, Gm, eps, Ri1, R1, nullptr);
    block_rmul(ctx, dtype, N, k, src, k, Ri1, 0.0, 1.0, dst, k);
    gram(ctx, dtype, N, k, dst, k, dst, k, Gm);
    small_cholqr(ctx, k, Gm, eps, Ri2, R2, nullptr);
    block_rmul(ctx, dtype, N, k, dst, k, Ri2, 0.0, 1.0, dst, k);
    small_gemm(ctx, k, R2, R1, 1.0, Rout);
  };

  // W -= sum_{i<=j} V_i (V_i^T W), the coefficients stored into (or, on the second pass, added to)
  // block column j of H.  Widths with multi-block kernels (k = 1, or 8..32 on the matrix cores) take
  // every projection from one pass over W and the update from another (classical Gram-Schmidt);
  // other widths project block by block.
  const bool mgs_mf = mf_eligible(k), mgs_dot = k == 1;
  const int mgs_max = mgs_mf ? mf_mgs_max_blocks(k) : mgs_dot ? mdot_max_blocks() : 1;
  const int KPm = mgs_dot ? 1 : (k <= 16 ? 16 : 32);
  const int64_t mslots = mgs_mf ? mf_mgram_slots(ctx, dtype, N, k) : mgs_dot ? mdot_slots(ctx, N) : 1;
  double* Cb = (mgs_mf || mgs_dot) ? ctx->ws.get<double>(pre + "_Cb", (size_t)(m + 1) * kk) : nullptr;
  double* mpart = (mgs_mf || mgs_dot)
                      ? ctx->ws.get<double>(pre + "_mpart", (size_t)mgs_max * KPm * KPm * mslots) : nullptr;
  const int64_t vstride = (int64_t)N * k;  // elements between consecutive basis blocks
  auto project = [&](int j, bool second) {
    if (!(mgs_mf || mgs_dot)) {
      for (int i = 0; i <= j; ++i) {
        gram(ctx, dtype, N, k, Vb(i), k, W, k, Hb);
        hblock(ctx, k, Hb, H, ldh, i * k, j * k, second);
        block_rmul(ctx, dtype, N, k, Vb(i), k, Hb, 1.0, -1.0, W, k);
      }
      return;
    }
    for (int i0 = 0; i0 <= j; i0 += mgs_max) {
      const int nb = std::min(mgs_max, j + 1 - i0);
      int ns = 0;
      if (mgs_mf)
        mf_mgram(ctx, dtype, N, k, nb, Vb(i0), vstride, W, mpart, &ns);
      else
        mdot(ctx, dtype, N, nb, Vb(i0), vstride, W, mpart, &ns);
      mf_mgs_finalize(ctx, mpart, ns, k, nb, Cb + (size_t)i0 * kk, H, ldh, i0 * k, j * k, second);
    }
    for (int i0 = 0; i0 <= j; i0 += mgs_max) {
      const int nb = std::min(mgs_max, j + 1 - i0);
      if (mgs_mf)
        mf_mrmul(ctx, dtype, N, k, nb, Vb(i0), vstride, Cb + (size_t)i0 * kk, W);
      else
        maxpy(ctx, dtype, N, nb, Vb(i0), vstride, Cb + (size_t)i0 * kk, W);
    }
  };

  ops.residual(B, X, x0_zero, W);
  colnorms2(ctx, dtype, N, k, W, k, nrmd);
  std::vector<double> nrm0, res;
  read_host(ctx, nrmd, k, nrm0);
  st = KrylovStats{};
  if (converged(nrm0, nrm0, rtol, &st.max_rel, true)) {
    st.converged = 1;
    return;
  }
  int total = 0;
  while (total < maxit) {
    cholqr2(W, Vb(0), S);  // R0 = V0 S
    BKTS_HIP(hipMemsetAsync(H, 0, sizeof(double) * hsz, ctx->stream));
    int jdone = 0;
    for (int j = 0; j < m && total < maxit; ++j) {
      ops.precond(Vb(j), Zb(j));
      ops.apply(Zb(j), W);  // W = A P V_j
      for (int pass = 0; pass < 2; ++pass) project(j, pass > 0);  // block Gram-Schmidt, twice
      cholqr2(W, Vb(j + 1), Tm);  // W = V_{j+1} H_{j+1,j}
      hblock(ctx, k, Tm, H, ldh, (j + 1) * k, j * k, false);
      gmres_qr_step(ctx, k, j, H, ldh, S, Rq, Vr, Br, Gq, resn);
      read_host(ctx, resn, k, res);
      ++total;
      jdone = j + 1;
      st.iterations = total;
      if (converged(res, nrm0, rtol, &st.max_rel, false)) break;
    }
    gmres_backsolve(ctx, k, jdone * k, Rq, ldh, Gq, lsq_eps, Y);
    BKTS_HIP(hipMemsetAsync(W, 0, blk, ctx->stream));
    if (ops.flexible) {  // X += sum_i (P V_i) Y_i
      for (int i = 0; i < jdone; ++i) block_rmul(ctx, dtype, N, k, Zb(i), k, Y + (size_t)i * kk, 1.0, 1.0, W, k);
      block_cast_scale(ctx, N, k, dtype, W, k, dtype, X, k, nullptr, false, true);
    } else {  // X += P sum_i V_i Y_i
      for (int i = 0; i < jdone; ++i) block_rmul(ctx, dtype, N, k, Vb(i), k, Y + (size_t)i * kk, 1.0, 1.0, W, k);
      ops.precond(W, Z);
      block_cast_scale(ctx, N, k, dtype, Z, k, dtype, X, k, nullptr, false, true);
    }
    // true residual for the next cycle (and the final check)
    ops.residual(B, X, false, W);
    colnorms2(ctx, dtype, N, k, W, k, nrmd);
    std::vector<double> nr;
    read_host(ctx, nrmd, k, nr);
    if (converged(nr, nrm0, rtol, &st.max_rel, true)) {
      st.converged = 1;
      return;
    }
  }
  st.converged = 0;
}

void block_gmres(bkts_ctx ctx, const bkts_op_s& op, int dtype, int k, double a, double b, const void* B, void* X,
                 bool x0_zero, bool jacobi, double rtol, int restart, int maxit, KrylovStats& st,
                 const bkts_op_s* mgop) {
  const int64_t N = op.N;
  const size_t blk = esize(dtype) * N * k;
  const double* dinv = nullptr;
  if (jacobi && !mgop) {
    double* d = ctx->ws.get<double>("gm_dinv", N);
    jacobi_inverse(ctx, op, a, b, d);
    dinv = d;
  }
  GmresOps ops;
  ops.apply = [&](const void* in, void* out) { spmm(ctx, op, dtype, k, 0.0, nullptr, k, a, in, k, b, out, k); };
  ops.precond = [&](const void* in, void* out) {  // right preconditioner: Jacobi, or one V-cycle (linear, fixed)
    if (mgop)
      mg_vcycle(ctx, *mgop, dtype, k, a, b, in, out);
    else
      scale_rows(ctx, dtype, N, k, dinv, in, out);
  };
  ops.residual = [&](const void* Bp, void* Xp, bool zero, void* Wp) {
    if (zero) {
      BKTS_HIP(hipMemsetAsync(Xp, 0, blk, ctx->stream));
      BKTS_HIP(hipMemcpyAsync(Wp, Bp, blk, hipMemcpyDeviceToDevice, ctx->stream));
    } else {
      spmm(ctx, op, dtype, k, 1.0, Bp, k, -a, Xp, k, -b, Wp, k);  // W = B - A X
    }
  };
  gmres_core(ctx, dtype, N, k, ops, B, X, x0_zero, rtol, restart, maxit, st);
}

// Vectorized BiCGStab: the k columns advance together through one block operator application per
// half step (the matrix streams once for all of them), each column with its own scalars alpha_j,
// omega_j, beta_j taken from the diagonals of the k x k products (the lane-wise form of a
// vectorized solver).  Coupling the columns through k x k solves (the block form) needs a
// well-conditioned residual block at every step, which FP32 windows of Algorithm 1 do not keep.
void block_bicgstab(bkts_ctx ctx, const bkts_op_s& op, int dtype, int k, double a, double b, const void* B, void* X,
                   bool x0_zero, bool jacobi, double rtol, int maxit, KrylovStats& st, const ColOp* cop,
                   const bkts_op_s* mgop) {
  const int64_t N = op.N;
  const size_t es = esize(dtype);
  const size_t blk = es * N * k;
  const std::string tag = dtype == BKTS_F64 ? "d" : "s";
  void* R = ctx->ws.get("bs_R_" + tag, blk);
  void* Rt = ctx->ws.get("bs_Rt_" + tag, blk);
  void* P = ctx->ws.get("bs_P_" + tag, blk);
  void* Ph = ctx->ws.get("bs_Ph_" + tag, blk);
  void* V = ctx->ws.get("bs_V_" + tag, blk);
  void* Sb = ctx->ws.get("bs_S_" + tag, blk);
  void* Sh = ctx->ws.get("bs_Sh_" + tag, blk);
  void* T = ctx->ws.get("bs_T_" + tag, blk);
  const size_t kk = (size_t)k * k;
  // per-column dots (k each): m1 = rt.v, mr = rt.r, ts = t.s, tt = t.t, m3 = rt.t; diagonal
  // coefficient matrices (k x k): alpha, beta, omega
  double* sm = ctx->ws.get<double>("bs_small", 3 * kk + 6 * k);
  double *al = sm, *be = al + kk, *W = be + kk;
  double *m1 = W + kk, *mr = m1 + k, *ts = mr + k, *tt = ts + k, *m3 = tt + k, *nrmd = m3 + k;
  const double* dinv = nullptr;
  if (jacobi && !mgop) {
    double* d = ctx->ws.get<double>("bs_dinv", N);
    jacobi_inverse(ctx, op, a, b, d);
    dinv = d;
  }
  // right preconditioner M^-1: the Jacobi scaling (fused into the update kernels), or one V-cycle of
  // the multigrid built from mgop for a I + b K_mg, applied after the kernel has formed the vector
  auto precondition = [&](const void* in, void* out) {
    if (mgop) mg_vcycle(ctx, *mgop, dtype, k, a, b, in, out);
  };
  // out = A in, column by column: one SpMM for K in, then each column's own a_j, b_j
  auto apply = [&](const void* in, void* out) {
    if (!cop) return spmm(ctx, op, dtype, k, 0.0, nullptr, k, a, in, k, b, out, k);
    spmm(ctx, op, dtype, k, 0.0, nullptr, k, 0.0, in, k, 1.0, out, k);
    col_affine(ctx, dtype, N, k, nullptr, in, out, cop->a, cop->b);
  };
  if (x0_zero) {
    BKTS_HIP(hipMemsetAsync(X, 0, blk, ctx->stream));
    BKTS_HIP(hipMemcpyAsync(R, B, blk, hipMemcpyDeviceToDevice, ctx->stream));
  } else if (!cop) {
    spmm(ctx, op, dtype, k, 1.0, B, k, -a, X, k, -b, R, k);
  } else {  // R = B - (a_j X_j + b_j K X_j)
    spmm(ctx, op, dtype, k, 0.0, nullptr, k, 0.0, X, k, 1.0, R, k);
    col_affine(ctx, dtype, N, k, B, X, R, cop->a, cop->b);
  }
  BKTS_HIP(hipMemcpyAsync(Rt, R, blk, hipMemcpyDeviceToDevice, ctx->stream));
  BKTS_HIP(hipMemcpyAsync(P, R, blk, hipMemcpyDeviceToDevice, ctx->stream));
  colnorms2(ctx, dtype, N, k, R, k, nrmd);
  std::vector<double> nrm0, nrm;
  read_host(ctx, nrmd, k, nrm0);
  st = KrylovStats{};
  if (converged(nrm0, nrm0, rtol, &st.max_rel, true)) {
    st.converged = 1;
    return;
  }
  if (mgop)
    precondition(P, Ph);
  else
    scale_rows(ctx, dtype, N, k, dinv, P, Ph);
  // Convergence is read one iteration late: the norms of iteration it land in pinned host memory
  // behind an event, and the host reads them after it has enqueued the residual half of iteration
  // it + 1, before that iteration's X update, so the iterates are those of a synchronous check.
  // The X update skips every column whose new residual norm is not finite (a breakdown keeps the
  // last finite iterate).
  double* hbuf = ctx->host_stage(2 * k);
  ctx->sync();
  double* hbuf_dev = nullptr;
  BKTS_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&hbuf_dev), hbuf, 0));
  hipEvent_t ev[2];
  BKTS_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming | hipEventDisableSystemFence));
  BKTS_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming | hipEventDisableSystemFence));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() { (void)hipEventDestroy(e[0]); (void)hipEventDestroy(e[1]); }
  } guard{ev};
  auto check = [&](int it) -> int {  // 1 = converged, -1 = breakdown, 0 = continue
    BKTS_HIP(hipEventSynchronize(ev[it & 1]));
    const double* h = hbuf + (it & 1) * k;
    nrm.assign(h, h + k);
    for (double v : nrm)
      if (!std::isfinite(v)) return -1;
    st.iterations = it;
    return converged(nrm, nrm0, rtol, &st.max_rel, true) ? 1 : 0;
  };
  auto finish = [&](int state) {
    ctx->sync();  // the residual half of the next iteration is in flight; it does not touch X
    st.breakdown = state == -1 ? 1 : 0;
    st.converged = state == 1 ? 1 : 0;
  };
  for (int it = 1; it <= maxit; ++it) {
    apply(Ph, V);  // V = A D^-1 P
    {
      const void* xs[2] = {Rt, Rt};
      const void* ys[2] = {V, R};
      double* os[2] = {m1, mr};
      col_dots(ctx, dtype, N, k, 2, xs, ys, os);
    }
    small_diag_ratio(ctx, k, mr, m1, 1.0, al);           // alpha_j = (rt_j^T r_j) / (rt_j^T v_j)
    bicg_s_step(ctx, dtype, N, k, R, V, al, dinv, Sb, Sh);  // S = R - V alpha, Sh = D^-1 S
    precondition(Sb, Sh);
    apply(Sh, T);  // T = A D^-1 S
    {
      const void* xs[3] = {T, T, Rt};
      const void* ys[3] = {Sb, T, T};
      double* os[3] = {ts, tt, m3};
      col_dots(ctx, dtype, N, k, 3, xs, ys, os);
    }
    small_diag_ratio(ctx, k, ts, tt, 1.0, W);  // omega_j = (t_j^T s_j) / (t_j^T t_j)
    bicg_r_step(ctx, dtype, N, k, Sb, T, W, R);  // R = S - T omega
    colnorms2(ctx, dtype, N, k, R, k, nrmd);
    publish(ctx, nrmd, k, hbuf_dev + (it & 1) * k);
    BKTS_HIP(hipEventRecord(ev[it & 1], ctx->stream));
    if (it > 1) {  // iteration it - 1 is complete: stop there if it converged or broke down
      const int state = check(it - 1);
      if (state != 0) {
        finish(state);  // this iteration's residual work is dropped, X is that of it - 1
        return;
      }
    }
    bicg_x_step(ctx, dtype, N, k, Ph, Sh, al, W, nrmd, X);  // X += D^-1 P alpha + D^-1 S omega
    small_diag_ratio(ctx, k, m3, m1, -1.0, be);  // beta_j = -(rt_j^T t_j) / (rt_j^T v_j)
    bicg_p_step(ctx, dtype, N, k, R, V, W, be, dinv, P, Ph);  // P = R + (P - V omega) beta, Ph = D^-1 P
    precondition(P, Ph);
  }
  finish(maxit >= 1 ? check(maxit) : 0);
}

}  // namespace bkts

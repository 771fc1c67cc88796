// Block Krylov solvers for (a I + b K) X = B on the device (block methods: Sec. 1,
// eq. basic-matrix-equation; block CG after O'Leary).  Every coefficient matrix is k x k FP64 and
// stays on the GPU; the host only reads the k column norms to decide convergence.
//
// Block CG in conjugate-direction form, with the Jacobi-preconditioned residual Z = D^-1 R:
//   Q = A P;  G = P^T Q;  alpha = G^+ gamma;  X += P alpha;  R -= Q alpha;
//   gamma = R^T Z;  T = Q^T Z;  beta = -G^+ T;  P = Z + P beta.
// G^+ is a truncated Cholesky inverse of the Jacobi-scaled G: directions that have become
// numerically dependent (columns that converged, duplicated columns after a pipelining shift)
// are dropped instead of breaking the iteration.
#include "krylov.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

#include "vecops.hpp"
#include "wide.hpp"

namespace bkts {

namespace {

struct Small {
  double *G, *gamma, *T, *alpha, *beta, *nrm, *nrm0;
  int* ndefl;
};

// Gram matrices inside the inner iteration: FP32 blocks of 5 or more columns use the FP32 matrix
// cores (per-tile FP32 sums, FP64 across tiles); everything else the exact-FP64 kernels.
void inner_gram(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, const void* Y, double* G) {
  if (wide_eligible(dtype, k))
    return w_gram(ctx, N, k, static_cast<const float*>(X), static_cast<const float*>(Y), G);
  gram(ctx, dtype, N, k, X, k, Y, k, G);
}

Small small_bufs(bkts_ctx ctx, const std::string& tag, int k) {
  const size_t kk = (size_t)k * k;
  double* base = ctx->ws.get<double>("small_" + tag, 5 * kk + 2 * k + 2);
  Small s;
  s.G = base;
  s.gamma = base + kk;
  s.T = base + 2 * kk;
  s.alpha = base + 3 * kk;
  s.beta = base + 4 * kk;
  s.nrm = base + 5 * kk;
  s.ndefl = reinterpret_cast<int*>(s.nrm + k);  // right after the norms: one read-back covers both
  s.nrm0 = s.nrm + k + 1;
  return s;
}

void read_norms(bkts_ctx ctx, const double* dev, int k, std::vector<double>& out, const int* ndefl_dev = nullptr,
                int* ndefl = nullptr) {
  double* h = ctx->host_stage(k + 1);
  BKTS_HIP(hipMemcpyAsync(h, dev, sizeof(double) * k, hipMemcpyDeviceToHost, ctx->stream));
  if (ndefl_dev)
    BKTS_HIP(hipMemcpyAsync(reinterpret_cast<int*>(h + k), ndefl_dev, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  ctx->sync();
  out.assign(h, h + k);
  if (ndefl && ndefl_dev) *ndefl = *reinterpret_cast<int*>(h + k);
}

bool all_converged(const std::vector<double>& nrm, const std::vector<double>& nrm0, double rtol, double* maxrel) {
  bool ok = true;
  double mr = 0.0;
  for (size_t j = 0; j < nrm.size(); ++j) {
    if (!std::isfinite(nrm[j])) throw Error{BKTS_EBREAKDOWN, fmt("non-finite residual in column %zu", j)};
    const double rel = nrm0[j] > 0.0 ? std::sqrt(nrm[j] / nrm0[j]) : (nrm[j] > 0.0 ? INFINITY : 0.0);
    mr = std::max(mr, rel);
    if (!(nrm[j] <= rtol * rtol * nrm0[j])) ok = false;
  }
  if (maxrel) *maxrel = mr;
  return ok;
}

}  // namespace

// Block CG on contiguous (ld = k) blocks of element type dtype.
void block_cg(bkts_ctx ctx, const bkts_op_s& op, int dtype, int k, double a, double b, const void* B, void* X,
              bool x0_zero, bool jacobi, double rtol, int maxit, KrylovStats& st) {
  const int64_t N = op.N;
  const size_t es = esize(dtype);
  const std::string tag = dtype == BKTS_F64 ? "d" : "s";
  void* R = ctx->ws.get("cg_R_" + tag, es * N * k);
  void* P = ctx->ws.get("cg_P_" + tag, es * N * k);
  void* Q = ctx->ws.get("cg_Q_" + tag, es * N * k);
  Small s = small_bufs(ctx, "cg" + tag, k);
  const double eps = cg_pivot_floor(dtype);
  const double* dK = nullptr;  // inverse Jacobi diagonal of a I + b K, computed once per solve
  if (jacobi) {
    double* d = ctx->ws.get<double>("cg_dinv", N);
    jacobi_inverse(ctx, op, a, b, d);
    dK = d;
  }

  if (x0_zero) {
    BKTS_HIP(hipMemsetAsync(X, 0, es * N * k, ctx->stream));
    BKTS_HIP(hipMemcpyAsync(R, B, es * N * k, hipMemcpyDeviceToDevice, ctx->stream));
  } else
    spmm(ctx, op, dtype, k, 1.0, B, k, -a, X, k, -b, R, k);
  colnorms2(ctx, dtype, N, k, R, k, s.nrm0);
  std::vector<double> nrm0, nrm;
  read_norms(ctx, s.nrm0, k, nrm0);
  st.iterations = 0;
  st.deflations = 0;
  st.converged = all_converged(nrm0, nrm0, rtol, &st.max_rel) ? 1 : 0;
  if (st.converged) return;

  cg_pupdate(ctx, dtype, N, k, P, R, nullptr, dK);
  inner_gram(ctx, dtype, N, k, R, P, s.gamma);
  // Convergence is read back one iteration late: the norms of iteration it are copied to pinned
  // memory behind an event while iteration it+1 is already enqueued, so the GPU never waits for
  // the host.  Stopping one iteration after the test passes only adds a valid CG step.
  double* hbuf = ctx->host_stage(2 * (k + 2));
  ctx->sync();
  hipEvent_t ev[2];
  BKTS_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  BKTS_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() { (void)hipEventDestroy(e[0]); (void)hipEventDestroy(e[1]); }
  } guard{ev};
  auto check = [&](int it) -> int {  // 1 = converged, -1 = all directions deflated, 0 = continue
    const int slot = it & 1;
    BKTS_HIP(hipEventSynchronize(ev[slot]));
    double* h = hbuf + slot * (k + 2);
    nrm.assign(h, h + k);
    const int nd = *reinterpret_cast<int*>(h + k);
    st.iterations = it;
    st.deflations = std::max(st.deflations, nd);
    if (all_converged(nrm, nrm0, rtol, &st.max_rel)) return 1;
    return nd >= k ? -1 : 0;
  };
  // k <= 4: each fold of partials and its k x k solve share one launch (five launches per
  // iteration instead of seven)
  // (for wider blocks the separate fold and solve launches measure faster: the fused form's
  // k x k working set per workgroup costs more than the launch it saves)
  const bool fused = rk_eligible(k);
  CgTail tail_sg, tail_up;
  if (fused) {
    tail_sg.counter = ctx->tail_counter(0);
    tail_sg.eps = eps;
    tail_sg.G = s.G;
    tail_sg.gamma_in = s.gamma;
    tail_sg.alpha = s.alpha;
    tail_sg.ndefl = s.ndefl;
    tail_up.counter = ctx->tail_counter(1);
    tail_up.eps = eps;
    tail_up.G = s.G;
    tail_up.gamma = s.gamma;
    tail_up.T = s.T;
    tail_up.nrm = s.nrm;
    tail_up.beta = s.beta;
    tail_up.ndefl = s.ndefl;  // read only: copied to the host next to the norms
  }
  // the fused tail writes the norms straight into the pinned staging buffer (no copy launch)
  double* hbuf_dev = nullptr;
  if (fused) BKTS_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&hbuf_dev), hbuf, 0));
  int restarts = 0;
  for (int it = 1; it <= maxit; ++it) {
    if (fused) {
      rk_spmm_gram(ctx, op, dtype, k, a, P, b, Q, s.G, &tail_sg);  // also alpha = G^+ gamma
    } else {
      spmm(ctx, op, dtype, k, 0.0, nullptr, k, a, P, k, b, Q, k);
      inner_gram(ctx, dtype, N, k, P, Q, s.G);
    }
    const int slot = it & 1;
    if (fused) {
      tail_up.host = hbuf_dev + slot * (k + 2);
      rk_cg_update(ctx, dtype, N, k, X, P, R, Q, s.alpha, dK, s.gamma, s.T, s.nrm, &tail_up);  // also beta
    } else {
      small_spd_solve(ctx, k, s.G, s.gamma, 1.0, eps, s.alpha, s.ndefl);
      cg_update(ctx, dtype, N, k, X, P, R, Q, s.alpha, dK, s.gamma, s.T, s.nrm);
      BKTS_HIP(hipMemcpyAsync(hbuf + slot * (k + 2), s.nrm, sizeof(double) * (k + 1), hipMemcpyDeviceToHost,
                              ctx->stream));
    }
    BKTS_HIP(hipEventRecord(ev[slot], ctx->stream));
    int state = 0;
    if (it > 1) state = check(it - 1);
    if (state == 1) {
      ctx->sync();  // iteration `it` is in flight; it only improves X
      st.iterations = it;
      st.converged = 1;
      return;
    }
    if (state == -1) {  // every search direction collapsed: restart from the preconditioned residual
      if (++restarts > 3) throw Error{BKTS_EBREAKDOWN, "block CG: search space collapsed repeatedly"};
      cg_pupdate(ctx, dtype, N, k, P, R, nullptr, dK);
      inner_gram(ctx, dtype, N, k, R, P, s.gamma);
      continue;
    }
    restarts = 0;
    if (!fused) small_spd_solve(ctx, k, s.G, s.T, -1.0, eps, s.beta, nullptr);
    cg_pupdate(ctx, dtype, N, k, P, R, s.beta, dK);
  }
  if (check(maxit) == 1) {
    st.converged = 1;
    return;
  }
  st.converged = 0;
}

// Block CG preconditioned by the multigrid V-cycle (mg.hip).  Z = M^-1 R is a block of its own, so
// gamma = R^T Z and T = Q^T Z are separate Gram passes (the Jacobi form folds them into the update);
// the deflating k x k solves and the restart on a collapsed search space are those of block_cg.
void block_pcg_mg(bkts_ctx ctx, const bkts_op_s& op, int dtype, int k, double a, double b, const void* B, void* X,
                  bool x0_zero, double rtol, int maxit, KrylovStats& st, const SolveHints* hints) {
  const int64_t N = op.N;
  const size_t es = esize(dtype);
  const std::string tag = dtype == BKTS_F64 ? "d" : "s";
  // with a zero initial guess and a scratch right-hand side, B itself becomes the residual block
  const bool take_b = x0_zero && hints && hints->b_scratch;
  void* R = take_b ? const_cast<void*>(B) : ctx->ws.get("mgcg_R_" + tag, es * N * k);
  void* P = ctx->ws.get("mgcg_P_" + tag, es * N * k);
  void* Q = ctx->ws.get("mgcg_Q_" + tag, es * N * k);
  void* Z = ctx->ws.get("mgcg_Z_" + tag, es * N * k);
  Small s = small_bufs(ctx, "mgcg" + tag, k);
  const double eps = cg_pivot_floor(dtype);
  const bool rowk = rk_eligible(k);
  // k <= 4 on a hierarchy with a separate finest prolongation: the V-cycle's last pass folds
  // gamma = R^T Z, T = Q^T Z and the norms of R, one launch folds those partials and solves for beta
  // (writing the norms and the deflation count to pinned host memory), and the Gram of the SpMM pass
  // is folded and solved for alpha in one launch: 12 launches per iteration instead of 20.  The
  // update is split: R -= Q alpha feeds the V-cycle, and X += P alpha joins the direction update
  // P = Z + P beta after it, in one pass that reads the old P once for both.
  const bool fused = rowk && mg_fusable(ctx, op, k);
  // from zero, the fused form's first direction update writes X = P alpha, so X is not cleared
  // (a return before that update clears it)
  bool x_pending = x0_zero && fused;
  auto clear_x = [&]() {
    if (x_pending) BKTS_HIP(hipMemsetAsync(X, 0, es * N * k, ctx->stream));
    x_pending = false;
  };
  if (x0_zero) {
    if (!fused) BKTS_HIP(hipMemsetAsync(X, 0, es * N * k, ctx->stream));
    if (!take_b) BKTS_HIP(hipMemcpyAsync(R, B, es * N * k, hipMemcpyDeviceToDevice, ctx->stream));
  } else {
    spmm(ctx, op, dtype, k, 1.0, B, k, -a, X, k, -b, R, k);
  }
  std::vector<double> nrm0, nrm;
  if (x0_zero && hints && hints->nrm0) {  // the caller knows the squared column norms of B
    nrm0.assign(hints->nrm0, hints->nrm0 + k);
  } else {
    colnorms2(ctx, dtype, N, k, R, k, s.nrm0);
    read_norms(ctx, s.nrm0, k, nrm0);
  }
  st.iterations = 0;
  st.deflations = 0;
  st.converged = all_converged(nrm0, nrm0, rtol, &st.max_rel) ? 1 : 0;
  if (st.converged) {
    clear_x();
    return;
  }
  auto precondition = [&]() {  // P = Z = M^-1 R (the cycle writes the first direction directly), gamma = R^T P
    if (fused) {  // gamma from the finest prolongation's reductions (R in Q's place; T and the norms unused)
      MgFuse fu;
      fu.Q = R;
      mg_vcycle(ctx, op, dtype, k, a, b, R, P, &fu);
      BKTS_REQUIRE(fu.nslots > 0, "multigrid: the fused reductions were not produced");
      finalize_gram(ctx, fu.partials, (int)fu.nslots, k, k, s.gamma);
    } else {
      mg_vcycle(ctx, op, dtype, k, a, b, R, P);
      inner_gram(ctx, dtype, N, k, R, P, s.gamma);
    }
  };
  precondition();
  // Convergence is read one iteration late, as in block_cg: the norms of iteration it are copied to
  // pinned memory behind an event while iteration it+1 is enqueued.  No read-back into the staging
  // buffer is pending here (every earlier one was waited for, and a fused solve leaves none in
  // flight), so the first V-cycle runs on while the loop is set up.
  double* hbuf = ctx->host_stage(2 * (k + 2));
  hipEvent_t ev[2];
  // The kernels write the norms and the deflation count straight into coherent pinned memory, so the
  // events that pace the host need no system-scope fence (which would write back the whole L2 once
  // per iteration).
  BKTS_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming | hipEventDisableSystemFence));
  BKTS_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming | hipEventDisableSystemFence));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() { (void)hipEventDestroy(e[0]); (void)hipEventDestroy(e[1]); }
  } guard{ev};
  auto check = [&](int it) -> int {  // 1 = converged, -1 = all directions deflated, 0 = continue
    const int slot = it & 1;
    BKTS_HIP(hipEventSynchronize(ev[slot]));
    double* h = hbuf + slot * (k + 2);
    nrm.assign(h, h + k);
    const int nd = *reinterpret_cast<int*>(h + k);
    st.iterations = it;
    st.deflations = std::max(st.deflations, nd);
    if (all_converged(nrm, nrm0, rtol, &st.max_rel)) return 1;
    return nd >= k ? -1 : 0;
  };
  CgTail tail_sg, tail_up;
  if (fused) {
    tail_sg.counter = ctx->tail_counter(0);
    tail_sg.eps = eps;
    tail_sg.G = s.G;
    tail_sg.gamma_in = s.gamma;
    tail_sg.alpha = s.alpha;
    tail_sg.ndefl = s.ndefl;
    tail_up.counter = ctx->tail_counter(1);
    tail_up.eps = eps;
    tail_up.G = s.G;
    tail_up.gamma = s.gamma;
    tail_up.T = s.T;
    tail_up.nrm = s.nrm;
    tail_up.beta = s.beta;
    tail_up.ndefl = s.ndefl;  // read only: copied to the host next to the norms
  }
  // the norms and the deflation count are written straight into the pinned buffer (no copy launch)
  double* hbuf_dev = nullptr;
  BKTS_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&hbuf_dev), hbuf, 0));
  int restarts = 0;
  for (int it = 1; it <= maxit; ++it) {
    const int slot = it & 1;
    double* hn = hbuf_dev + slot * (k + 2);
    if (fused) {
      rk_spmm_gram(ctx, op, dtype, k, a, P, b, Q, s.G, &tail_sg);  // also alpha = G^+ gamma
      rk_cg_r_update(ctx, dtype, N, k, R, Q, s.alpha);
    } else {
      if (rowk) {  // Q = a P + b K P with G = P^T Q folded from the same pass
        rk_spmm_gram(ctx, op, dtype, k, a, P, b, Q, s.G, nullptr);
      } else {
        spmm(ctx, op, dtype, k, 0.0, nullptr, k, a, P, k, b, Q, k);
        inner_gram(ctx, dtype, N, k, P, Q, s.G);
      }
      small_spd_solve(ctx, k, s.G, s.gamma, 1.0, eps, s.alpha, reinterpret_cast<int*>(hn + k));
      // X += P alpha, R -= Q alpha and the norms of R (its gamma and T outputs are recomputed below)
      cg_update(ctx, dtype, N, k, X, P, R, Q, s.alpha, nullptr, s.T, s.beta, hn);
      BKTS_HIP(hipEventRecord(ev[slot], ctx->stream));
    }
    // the norms of iteration it-1 (in the fused form they come after its V-cycle, which the GPU
    // finished before starting this iteration's SpMM)
    const int state = it > 1 ? check(it - 1) : 0;
    // this iteration's X += P alpha on its own when no direction update follows
    if (fused && state != 0) rk_cg_x_update(ctx, dtype, N, k, X, P, s.alpha);
    if (state == 1) {
      // iteration `it` is in flight and only improves X; the caller's next kernels follow it on the
      // stream.  The fused form has no event or read-back of this iteration outstanding, so it
      // returns at once; the other form waits for the norms it records into the staging buffer.
      if (!fused) ctx->sync();
      st.iterations = it;
      st.converged = 1;
      return;
    }
    if (state == -1) {  // every search direction collapsed: restart from the preconditioned residual
      if (++restarts > 3) throw Error{BKTS_EBREAKDOWN, "block CG: search space collapsed repeatedly"};
      precondition();
      if (fused) {  // this iteration's norms, for the check of the next one (copied, then a full sync)
        colnorms2(ctx, dtype, N, k, R, k, s.nrm);
        BKTS_HIP(hipMemcpyAsync(hbuf + slot * (k + 2), s.nrm, sizeof(double) * k, hipMemcpyDeviceToHost,
                                ctx->stream));
        BKTS_HIP(hipMemcpyAsync(reinterpret_cast<int*>(hbuf + slot * (k + 2) + k), s.ndefl, sizeof(int),
                                hipMemcpyDeviceToHost, ctx->stream));
        BKTS_HIP(hipEventRecord(ev[slot], ctx->stream));
        ctx->sync();
      }
      continue;
    }
    restarts = 0;
    if (fused) {
      MgFuse fu;
      fu.Q = Q;
      mg_vcycle(ctx, op, dtype, k, a, b, R, Z, &fu);
      BKTS_REQUIRE(fu.nslots > 0, "multigrid: the fused reductions were not produced");
      tail_up.host = hn;
      fold_solve(ctx, 1, k, k, fu.partials, fu.nslots, tail_up);  // gamma, T, nrm, then beta = -G^+ T
      BKTS_HIP(hipEventRecord(ev[slot], ctx->stream));
      rk_cg_xp_update(ctx, dtype, N, k, X, P, Z, s.alpha, s.beta, x_pending);  // X += P alpha; P = Z + P beta
      x_pending = false;
      continue;
    } else {
      mg_vcycle(ctx, op, dtype, k, a, b, R, Z);
      if (rowk) {
        rk_gram2(ctx, dtype, N, k, R, Q, Z, s.gamma, s.T);  // gamma = R^T Z and T = Q^T Z in one pass
      } else {
        inner_gram(ctx, dtype, N, k, R, Z, s.gamma);
        inner_gram(ctx, dtype, N, k, Q, Z, s.T);
      }
      small_spd_solve(ctx, k, s.G, s.T, -1.0, eps, s.beta, nullptr);
    }
    cg_pupdate(ctx, dtype, N, k, P, Z, s.beta, nullptr);
  }
  clear_x();  // maxit < 1: no direction update ran
  if (check(maxit) == 1) {
    st.converged = 1;
    return;
  }
  st.converged = 0;
}

// One FP32 block CG solve of (a I + b K) V = R64 for FP64 blocks: R64 is scaled per column to
// unit norm, cast to FP32, solved to `rtol`, and the FP32 correction is scaled back and added to
// V64 (which need not be zero).
// The operator the multigrid preconditioner of a GMRES or BiCGStab solve is built from, or null
// without BKTS_PREC_MG.
static const bkts_op_s* mg_op(bkts_ctx ctx, const bkts_op_s& op, const bkts_solve_opts& o, const ColOp* cop) {
  if (o.precond != BKTS_PREC_MG) return nullptr;
  BKTS_REQUIRE(!cop, "multigrid does not precondition per-column operators");
  const bkts_op_s* m = mg_source(ctx, op);
  BKTS_REQUIRE(m, "multigrid needs the stencil form (BKTS_FMT_STENCIL) or a Newton Jacobian on a grid");
  return m;
}

// Dispatch on the Krylov method of the options.
static void krylov_run(bkts_ctx ctx, const bkts_op_s& op, const bkts_solve_opts& o, int dtype, int k, double a,
                       double b, const void* B, void* X, bool x0_zero, double rtol, int maxit, KrylovStats& st,
                       const ColOp* cop = nullptr, const SolveHints* hints = nullptr) {
  const bool jacobi = o.precond == BKTS_PREC_JACOBI;
  BKTS_REQUIRE(!cop || o.krylov == BKTS_BICGSTAB, "per-column operators need the vectorized BiCGStab");
  BKTS_REQUIRE(o.precond >= BKTS_PREC_NONE && o.precond <= BKTS_PREC_MG, "unknown preconditioner %d", o.precond);
  switch (o.krylov) {
    case BKTS_CG:
      if (o.precond == BKTS_PREC_MG)
        block_pcg_mg(ctx, op, dtype, k, a, b, B, X, x0_zero, rtol, maxit, st, hints);
      else
        block_cg(ctx, op, dtype, k, a, b, B, X, x0_zero, jacobi, rtol, maxit, st);
      break;
    case BKTS_GMRES:
      block_gmres(ctx, op, dtype, k, a, b, B, X, x0_zero, jacobi, rtol, o.restart, maxit, st, mg_op(ctx, op, o, cop));
      break;
    case BKTS_BICGSTAB:
      block_bicgstab(ctx, op, dtype, k, a, b, B, X, x0_zero, jacobi, rtol, maxit, st, cop, mg_op(ctx, op, o, cop));
      break;
    default: throw Error{BKTS_EINVAL, fmt("unknown Krylov method %d", o.krylov)};
  }
}

void f32_correction(bkts_ctx ctx, const bkts_op_s& op, const bkts_solve_opts& o, int k, double a, double b,
                    const double* R64, const double* n2_dev, const double* n2_host, double* V64, double coef,
                    double rtol, int maxit, KrylovStats& st, const ColOp* cop = nullptr) {
  const int64_t N = op.N;
  float* R32 = ctx->ws.get<float>("f32_R", (size_t)N * k);
  float* V32 = ctx->ws.get<float>("f32_V", (size_t)N * k);
  // column j scaled by 1 / ||R64_j|| (1 for a zero column), so the FP32 block has unit columns
  block_cast_scale(ctx, N, k, BKTS_F64, R64, k, BKTS_F32, R32, k, n2_dev, true, false, true);
  SolveHints h;
  h.b_scratch = true;  // R32 is this pass's own: the solver may take it as its residual block
  std::vector<double> n0(k);
  for (int j = 0; j < k; ++j) n0[j] = n2_host[j] > 0.0 ? 1.0 : 0.0;
  h.nrm0 = n0.data();
  krylov_run(ctx, op, o, BKTS_F32, k, a, b, R32, V32, true, rtol, maxit, st, cop, &h);
  block_cast_scale(ctx, N, k, BKTS_F32, V32, k, BKTS_F64, V64, k, n2_dev, false, true, true, coef);
}

void correct_f32(bkts_ctx ctx, const bkts_op_s& op, double a, double b, int k, const double* R, const double* rn2_dev,
                 const double* rn2_host, double coef, double* Y, const bkts_solve_opts& o, KrylovStats& st,
                 const ColOp* cop) {
  BKTS_REQUIRE(o.precision == BKTS_PRECISION_F32_REFINE, "correct_f32 needs FP32 inner solves");
  const int maxit = o.maxit > 0 ? o.maxit : 10000;
  const double inner = o.inner_rtol > 0.0 ? o.inner_rtol : 1e-4;
  st = KrylovStats{};
  f32_correction(ctx, op, o, k, a, b, R, rn2_dev, rn2_host, Y, coef, std::max(o.rtol, inner), maxit, st, cop);
  st.refinements = 1;
}

void solve(bkts_ctx ctx, const bkts_op_s& op, double a, double b, int k, const double* B, double* X, bool x0_zero,
           const bkts_solve_opts& o, bool single_f32_pass, KrylovStats& st, const ColOp* cop) {
  const int maxit = o.maxit > 0 ? o.maxit : 10000;
  if (o.precision == BKTS_PRECISION_F64) {
    krylov_run(ctx, op, o, BKTS_F64, k, a, b, B, X, x0_zero, o.rtol, maxit, st, cop);
    st.refinements = 0;
    return;
  }
  BKTS_REQUIRE(o.precision == BKTS_PRECISION_F32_REFINE, "unknown precision %d", o.precision);
  BKTS_REQUIRE(!cop || single_f32_pass, "per-column operators: FP64, or one FP32 pass inside the caller's loop");
  const int64_t N = op.N;
  const double inner = o.inner_rtol > 0.0 ? o.inner_rtol : 1e-4;
  double* n2 = ctx->ws.get<double>("ref_n2", k);
  if (single_f32_pass) {
    // the caller's outer loop supplies FP64 residuals: one scaled FP32 correction of X = 0
    BKTS_REQUIRE(x0_zero, "single FP32 pass needs a zero initial guess");
    BKTS_HIP(hipMemsetAsync(X, 0, sizeof(double) * N * k, ctx->stream));
    colnorms2(ctx, BKTS_F64, N, k, B, k, n2);
    std::vector<double> nb;
    read_norms(ctx, n2, k, nb);
    st = KrylovStats{};
    f32_correction(ctx, op, o, k, a, b, B, n2, nb.data(), X, 1.0, std::max(o.rtol, inner), maxit, st, cop);
    st.refinements = 1;
    return;
  }
  double* R64 = ctx->ws.get<double>("ref_R", (size_t)N * k);
  if (x0_zero) {
    BKTS_HIP(hipMemsetAsync(X, 0, sizeof(double) * N * k, ctx->stream));
    BKTS_HIP(hipMemcpyAsync(R64, B, sizeof(double) * N * k, hipMemcpyDeviceToDevice, ctx->stream));
  } else {
    spmm(ctx, op, BKTS_F64, k, 1.0, B, k, -a, X, k, -b, R64, k);
  }
  colnorms2(ctx, BKTS_F64, N, k, R64, k, n2);
  std::vector<double> nrm0, nrm;
  read_norms(ctx, n2, k, nrm0);
  nrm = nrm0;
  st = KrylovStats{};
  int total = 0;
  for (int ref = 0; ref < 60; ++ref) {
    if (all_converged(nrm, nrm0, o.rtol, &st.max_rel)) {
      st.converged = 1;
      return;
    }
    KrylovStats in;
    f32_correction(ctx, op, o, k, a, b, R64, n2, nrm.data(), X, 1.0, inner, maxit - total, in);
    total += in.iterations;
    st.iterations = total;
    st.refinements = ref + 1;
    st.deflations = std::max(st.deflations, in.deflations);
    spmm(ctx, op, BKTS_F64, k, 1.0, B, k, -a, X, k, -b, R64, k);
    colnorms2(ctx, BKTS_F64, N, k, R64, k, n2);
    read_norms(ctx, n2, k, nrm);
    if (total >= maxit) break;
  }
  st.converged = all_converged(nrm, nrm0, o.rtol, &st.max_rel) ? 1 : 0;
}

}  // namespace bkts

// extern "C" entry points: argument validation, exception-to-status mapping, dispatch.
#include <cmath>
#include <cstring>

#include "accel.hpp"
#include "advance.hpp"
#include <algorithm>

#include "internal.hpp"
#include "krylov.hpp"
#include "server.hpp"
#include "timecoupling.hpp"
#include "vecops.hpp"

namespace bkts {
bkts_op fv_assemble(bkts_ctx ctx, const bkts_grid* grid, const bkts_fv_coeffs* c, int format);
bkts_op op_from_csr(bkts_ctx ctx, int64_t N, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                    const double* val, int format);
void upload_window(bkts_ctx ctx, const bkts_tc_s& tc, int phase, int off, double* A1p, double* A2p, double* rsp);
const char* last_error();
}  // namespace bkts

using bkts::Error;

#define BKTS_API_BEGIN try {
#define BKTS_API_END                                                 \
  return BKTS_OK;                                                    \
  }                                                                  \
  catch (const Error& e) {                                           \
    bkts::set_last_error(e.msg);                                     \
    return e.status;                                                 \
  }                                                                  \
  catch (const std::exception& e) {                                  \
    bkts::set_last_error(std::string("internal error: ") + e.what()); \
    return BKTS_EDEVICE;                                             \
  }                                                                  \
  catch (...) {                                                      \
    bkts::set_last_error("unknown internal error");                  \
    return BKTS_EDEVICE;                                             \
  }

namespace {

void check_ctx(bkts_ctx ctx) { BKTS_REQUIRE(ctx, "ctx must not be NULL"); }

void check_block(const void* p, int k, int ld, const char* name) {
  BKTS_REQUIRE(p, "%s must not be NULL", name);
  BKTS_REQUIRE(ld >= k, "%s: leading dimension %d < k = %d", name, ld, k);
}

void check_k(int k) { BKTS_REQUIRE(k >= 1 && k <= BKTS_MAX_K, "k must be in 1..%d (got %d)", BKTS_MAX_K, k); }

void set_device(bkts_ctx ctx) { BKTS_HIP(hipSetDevice(ctx->device)); }

}  // namespace

extern "C" {

const char* bkts_last_error(void) { return bkts::last_error(); }
const char* bkts_version(void) { return "bkts 0.1 (gfx950)"; }

bkts_status bkts_ctx_create(int device, void* hip_stream, bkts_ctx* out) {
  BKTS_API_BEGIN
  BKTS_REQUIRE(out, "out must not be NULL");
  *out = nullptr;
  int ndev = 0;
  BKTS_HIP(hipGetDeviceCount(&ndev));
  BKTS_REQUIRE(device >= 0 && device < ndev, "device %d out of range (%d devices)", device, ndev);
  BKTS_HIP(hipSetDevice(device));
  bkts_ctx c = new bkts_ctx_s();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
    c->num_cu = ncu;
  try {
    bkts::scratch_init(device);  // this device's address of the allocation-free entry point's array
  } catch (...) {
    delete c;
    throw;
  }
  *out = c;
  BKTS_API_END
}

void bkts_ctx_destroy(bkts_ctx ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->ws.bufs.clear();
  if (ctx->h_pinned) (void)hipHostFree(ctx->h_pinned);
  delete ctx;
}

bkts_status bkts_ctx_synchronize(bkts_ctx ctx) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  ctx->sync();
  BKTS_API_END
}

bkts_status bkts_fv_assemble(bkts_ctx ctx, const bkts_grid* grid, const bkts_fv_coeffs* coeffs, int format,
                             bkts_op* out) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  BKTS_REQUIRE(out, "out must not be NULL");
  *out = nullptr;
  set_device(ctx);
  *out = bkts::fv_assemble(ctx, grid, coeffs, format);
  BKTS_API_END
}

bkts_status bkts_op_create_csr(bkts_ctx ctx, int64_t N, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                               const double* val, int format, bkts_op* out) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  BKTS_REQUIRE(out, "out must not be NULL");
  *out = nullptr;
  set_device(ctx);
  *out = bkts::op_from_csr(ctx, N, nnz, rowptr, col, val, format);
  BKTS_API_END
}

bkts_status bkts_op_info(bkts_op op, int64_t* N, int64_t* nnz) {
  BKTS_API_BEGIN
  BKTS_REQUIRE(op, "op must not be NULL");
  if (N) *N = op->N;
  if (nnz) *nnz = op->nnz;
  BKTS_API_END
}

bkts_status bkts_op_export_csr(bkts_op op, int32_t* rowptr, int32_t* col, double* val, double* b) {
  BKTS_API_BEGIN
  BKTS_REQUIRE(op, "op must not be NULL");
  bkts_ctx ctx = op->ctx;
  set_device(ctx);
  auto d2h = [&](void* dst, const void* src, size_t bytes) {
    if (dst && bytes) BKTS_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, ctx->stream));
  };
  d2h(rowptr, op->rowptr.p, sizeof(int32_t) * (op->N + 1));
  d2h(col, op->col.p, sizeof(int32_t) * op->nnz);
  d2h(val, op->val.p, sizeof(double) * op->nnz);
  d2h(b, op->b.p, sizeof(double) * op->N);
  ctx->sync();
  BKTS_API_END
}

void bkts_op_destroy(bkts_op op) {
  if (!op) return;
  (void)hipSetDevice(op->ctx->device);
  (void)hipStreamSynchronize(op->ctx->stream);
  delete op;
}

bkts_status bkts_spmm(bkts_ctx ctx, bkts_op op, int dtype, int k, double alpha, double beta, const void* X, int ldx,
                      void* Y, int ldy) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  BKTS_REQUIRE(op && op->ctx == ctx, "op must belong to ctx");
  BKTS_REQUIRE(dtype == BKTS_F64 || dtype == BKTS_F32, "dtype must be BKTS_F64 or BKTS_F32");
  check_k(k);
  check_block(X, k, ldx, "X");
  check_block(Y, k, ldy, "Y");
  BKTS_REQUIRE(X != Y, "X and Y must not alias");
  set_device(ctx);
  bkts::spmm(ctx, *op, dtype, k, 0.0, nullptr, k, alpha, X, ldx, beta, Y, ldy);
  BKTS_API_END
}

bkts_status bkts_mg_apply(bkts_ctx ctx, bkts_op op, int dtype, int k, double a, double b, const void* F, int ldf,
                          void* Z, int ldz) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  BKTS_REQUIRE(op && op->ctx == ctx, "op must belong to ctx");
  BKTS_REQUIRE(dtype == BKTS_F64 || dtype == BKTS_F32, "dtype must be BKTS_F64 or BKTS_F32");
  check_k(k);
  BKTS_REQUIRE(F && Z, "F and Z must not be NULL");
  BKTS_REQUIRE(ldf == k && ldz == k, "F and Z must be contiguous (ld == k)");
  const size_t bytes = (size_t)op->N * k * (dtype == BKTS_F64 ? 8 : 4);
  const char* f = static_cast<const char*>(F);
  const char* z = static_cast<const char*>(Z);
  BKTS_REQUIRE(f + bytes <= z || z + bytes <= f, "F and Z must not overlap");
  BKTS_REQUIRE(reinterpret_cast<uintptr_t>(F) % 16 == 0 && reinterpret_cast<uintptr_t>(Z) % 16 == 0,
               "F and Z must be 16-byte aligned");
  BKTS_REQUIRE(std::isfinite(a) && std::isfinite(b) && a >= 0.0 && b > 0.0, "need a >= 0 and b > 0");
  set_device(ctx);
  if (op->N > 0) bkts::mg_vcycle(ctx, *op, dtype, k, a, b, F, Z);
  BKTS_API_END
}

bkts_status bkts_gram(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, int ldx, const void* Y, int ldy,
                      double* G) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  BKTS_REQUIRE(dtype == BKTS_F64 || dtype == BKTS_F32, "dtype must be BKTS_F64 or BKTS_F32");
  BKTS_REQUIRE(N >= 0, "N must be >= 0");
  check_k(k);
  check_block(X, k, ldx, "X");
  check_block(Y, k, ldy, "Y");
  BKTS_REQUIRE(G, "G must not be NULL");
  set_device(ctx);
  bkts::gram(ctx, dtype, N, k, X, ldx, Y, ldy, G);
  BKTS_API_END
}

bkts_status bkts_gram_noalloc(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, int ldx, const void* Y,
                              int ldy, double* G) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  BKTS_REQUIRE(dtype == BKTS_F64 || dtype == BKTS_F32, "dtype must be BKTS_F64 or BKTS_F32");
  BKTS_REQUIRE(N >= 0, "N must be >= 0");
  check_k(k);
  check_block(X, k, ldx, "X");
  check_block(Y, k, ldy, "Y");
  BKTS_REQUIRE(G, "G must not be NULL");
  set_device(ctx);
  bkts::gram_noalloc(ctx, dtype, N, k, X, ldx, Y, ldy, G);
  BKTS_API_END
}

bkts_status bkts_tc_create(bkts_ctx ctx, const bkts_tc_desc* desc, bkts_tc* out) {
  BKTS_API_BEGIN
  BKTS_REQUIRE(out, "out must not be NULL");
  *out = nullptr;
  *out = bkts::tc_create(ctx, desc);
  BKTS_API_END
}

bkts_status bkts_tc_get(bkts_tc tc, int phase, double* A1, double* A2, double* beta, int* k, int* m_impl) {
  BKTS_API_BEGIN
  BKTS_REQUIRE(tc, "tc must not be NULL");
  BKTS_REQUIRE(phase >= 0 && phase < tc->m_impl, "phase must be in 0..%d", tc->m_impl - 1);
  const size_t kk = (size_t)tc->k * tc->k;
  if (A1) std::memcpy(A1, tc->A1[phase].data(), sizeof(double) * kk);
  if (A2) std::memcpy(A2, tc->A2[phase].data(), sizeof(double) * kk);
  if (beta) *beta = tc_beta(*tc, phase);
  if (k) *k = tc->k;
  if (m_impl) *m_impl = tc->m_impl;
  BKTS_API_END
}

void bkts_tc_destroy(bkts_tc tc) { delete tc; }

bkts_status bkts_residual(bkts_ctx ctx, bkts_op op, bkts_tc tc, int phase, const double* Y, int ldy,
                          const double* B0, int ldb0, int nb0, double* R, int ldr, double* col_norms2) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  BKTS_REQUIRE(op && op->ctx == ctx && tc, "op must belong to ctx and tc must not be NULL");
  BKTS_REQUIRE(phase >= 0 && phase < tc->m_impl, "phase must be in 0..%d", tc->m_impl - 1);
  BKTS_REQUIRE(!tc->fully_implicit || phase == 0, "a fully implicit tableau's windows start at stage 0 (whole steps)");
  const int k = tc->k;
  check_block(Y, k, ldy, "Y");
  check_block(R, k, ldr, "R");
  BKTS_REQUIRE(Y != R, "Y and R must not alias");
  BKTS_REQUIRE(nb0 >= 0 && nb0 <= k && nb0 <= 8, "nb0 must be in 0..min(k, 8)");
  if (B0 && nb0 > 0) BKTS_REQUIRE(ldb0 >= nb0, "ldb0 < nb0");
  set_device(ctx);
  double* nrm = ctx->ws.get<double>("api_res_nrm", k);
  bkts::window_residual(ctx, *op, *tc, phase, 0, Y, ldy, B0, ldb0, B0 ? nb0 : 0, R, ldr, nrm);
  if (col_norms2) {
    BKTS_HIP(hipMemcpyAsync(col_norms2, nrm, sizeof(double) * k, hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
  }
  BKTS_API_END
}

bkts_status bkts_block_solve(bkts_ctx ctx, bkts_op op, double alpha, double beta, int k, const double* B, int ldb,
                             double* X, int ldx, const bkts_solve_opts* opts, bkts_solve_info* info) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  BKTS_REQUIRE(op && op->ctx == ctx, "op must belong to ctx");
  check_k(k);
  check_block(B, k, ldb, "B");
  check_block(X, k, ldx, "X");
  BKTS_REQUIRE(opts, "opts must not be NULL");
  BKTS_REQUIRE(opts->rtol > 0.0 && opts->rtol < 1.0, "rtol must be in (0, 1)");
  BKTS_REQUIRE(std::isfinite(alpha) && std::isfinite(beta), "alpha and beta must be finite");
  set_device(ctx);
  const int64_t N = op->N;
  // the solvers work on contiguous blocks; stage strided inputs
  const double* Bc = B;
  double* Xc = X;
  if (ldb != k) {
    double* t = ctx->ws.get<double>("api_B", (size_t)N * k);
    bkts::block_cast_scale(ctx, N, k, BKTS_F64, B, ldb, BKTS_F64, t, k, nullptr, false, false);
    Bc = t;
  }
  if (ldx != k) {
    Xc = ctx->ws.get<double>("api_X", (size_t)N * k);
    bkts::block_cast_scale(ctx, N, k, BKTS_F64, X, ldx, BKTS_F64, Xc, k, nullptr, false, false);
  }
  bkts::KrylovStats st;
  bkts_status result = BKTS_OK;
  try {
    bkts::solve(ctx, *op, alpha, beta, k, Bc, Xc, false, *opts, false, st);
  } catch (const Error& e) {
    if (e.status != BKTS_EBREAKDOWN) throw;
    bkts::set_last_error(e.msg);
    result = BKTS_EBREAKDOWN;
  }
  if (ldx != k) bkts::block_cast_scale(ctx, N, k, BKTS_F64, Xc, k, BKTS_F64, X, ldx, nullptr, false, false);
  ctx->sync();
  if (info) {
    info->iterations = st.iterations;
    info->refinements = st.refinements;
    info->converged = st.converged;
    info->deflations = st.deflations;
    info->max_rel_residual = st.max_rel;
  }
  if (result != BKTS_OK) return result;
  if (!st.converged) {
    bkts::set_last_error(bkts::fmt("block solve not converged after %d iterations (max rel. residual %.3e)",
                                   st.iterations, st.max_rel));
    return BKTS_ENOCONV;
  }
  BKTS_API_END
}

bkts_status bkts_advance(bkts_ctx ctx, bkts_op op, bkts_tc tc, double* y, int n_steps, const bkts_solve_opts* inner,
                         double outer_rtol, int max_outer, double* y_hist, bkts_step_cb cb, void* user,
                         bkts_run_info* info) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  BKTS_REQUIRE(op && op->ctx == ctx && tc, "op must belong to ctx and tc must not be NULL");
  BKTS_REQUIRE(y, "y must not be NULL");
  BKTS_REQUIRE(n_steps >= 0, "n_steps must be >= 0");
  BKTS_REQUIRE(inner, "inner options must not be NULL");
  BKTS_REQUIRE(inner->rtol > 0.0 && inner->rtol < 1.0, "inner rtol must be in (0, 1)");
  BKTS_REQUIRE(outer_rtol > 0.0 && outer_rtol < 1.0, "outer_rtol must be in (0, 1)");
  BKTS_REQUIRE(max_outer >= 1, "max_outer must be >= 1");
  set_device(ctx);
  return bkts::advance(ctx, op, tc, y, n_steps, *inner, outer_rtol, max_outer, y_hist, cb, user, info);
  BKTS_API_END
}

bkts_status bkts_window_solve(bkts_ctx ctx, bkts_op op, bkts_tc tc, int phase, const double* B0, int ldb0, int nb0,
                              double* Y, int method, const bkts_solve_opts* inner, double rtol, int restart,
                              int maxit, bkts_window_info* info) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  BKTS_REQUIRE(op && op->ctx == ctx && tc, "op must belong to ctx and tc must not be NULL");
  BKTS_REQUIRE(phase >= 0 && phase < tc->m_impl, "phase must be in 0..%d", tc->m_impl - 1);
  BKTS_REQUIRE(!tc->fully_implicit || phase == 0, "a fully implicit tableau's windows start at stage 0 (whole steps)");
  BKTS_REQUIRE(Y, "Y must not be NULL");
  BKTS_REQUIRE(method == BKTS_WINDOW_FGMRES || method == BKTS_WINDOW_SPLITTING, "unknown window method %d", method);
  BKTS_REQUIRE(inner, "inner options must not be NULL");
  BKTS_REQUIRE(inner->rtol > 0.0 && inner->rtol < 1.0, "inner rtol must be in (0, 1)");
  BKTS_REQUIRE(rtol > 0.0 && rtol < 1.0, "rtol must be in (0, 1)");
  BKTS_REQUIRE(restart >= 1 && maxit >= 1, "restart and maxit must be >= 1");
  const int k = tc->k;
  BKTS_REQUIRE(nb0 >= 0 && nb0 <= k && nb0 <= 8, "nb0 must be in 0..min(k, 8)");
  if (B0 && nb0 > 0) BKTS_REQUIRE(ldb0 >= nb0, "ldb0 < nb0");
  set_device(ctx);
  bkts::WindowStats ws;
  bkts::window_solve(ctx, *op, *tc, phase, B0, ldb0, nb0, Y, *inner, method, rtol, restart, maxit, ws);
  ctx->sync();
  if (info) {
    info->iterations = ws.iterations;
    info->inner_iterations = ws.inner_iterations;
    info->precond_applications = ws.precond_applications;
    info->converged = ws.converged;
    info->rel_residual = ws.rel_residual;
  }
  if (!ws.converged) {
    bkts::set_last_error(bkts::fmt("window not converged after %d iterations (rel. residual %.3e)", ws.iterations,
                                   ws.rel_residual));
    return BKTS_ENOCONV;
  }
  BKTS_API_END
}

bkts_status bkts_profile_enable(bkts_ctx ctx, int enable) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  ctx->sync();
  ctx->prof.resolve();
  ctx->prof.reset();
  BKTS_REQUIRE(enable >= 0, "enable must be >= 0");
  ctx->prof.enabled = enable != 0;
  ctx->prof.period = enable > 1 ? enable : 1;
  BKTS_API_END
}

bkts_status bkts_profile_query(bkts_ctx ctx, int kernel, int64_t* launches, double* total_ms, double* bytes) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  BKTS_REQUIRE(kernel >= 0 && kernel < BKTS_K_COUNT, "kernel id out of range");
  ctx->sync();
  ctx->prof.resolve();
  const auto& a = ctx->prof.acc[kernel];
  if (launches) *launches = a.launches;
  if (total_ms) *total_ms = a.ms;
  if (bytes) *bytes = a.bytes;
  BKTS_API_END
}

bkts_status bkts_profile_samples(bkts_ctx ctx, int kernel, float* ms, int max, int* n) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  BKTS_REQUIRE(kernel >= 0 && kernel < BKTS_K_COUNT, "kernel id out of range");
  BKTS_REQUIRE(n && (ms || max == 0) && max >= 0, "need n, and ms unless max == 0");
  ctx->sync();
  ctx->prof.resolve();
  const auto& v = ctx->prof.acc[kernel].samples;
  const int m = (int)std::min<size_t>(v.size(), (size_t)max);
  for (int i = 0; i < m; ++i) ms[i] = v[i];
  *n = (int)v.size();
  BKTS_API_END
}

bkts_status bkts_stepper_create(bkts_ctx ctx, bkts_op op, bkts_tc tc, const double* y0, bkts_stepper* out) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  BKTS_REQUIRE(out, "out must not be NULL");
  *out = nullptr;
  BKTS_REQUIRE(op && op->ctx == ctx && tc, "op must belong to ctx and tc must not be NULL");
  BKTS_REQUIRE(y0, "y0 must not be NULL");
  set_device(ctx);
  *out = new bkts_stepper_s(ctx, op, tc, y0);
  BKTS_API_END
}

bkts_status bkts_stepper_advance(bkts_stepper st, int n_steps, const bkts_solve_opts* inner, double outer_rtol,
                                 int max_outer, double* y_hist, bkts_step_cb cb, void* user, bkts_run_info* info) {
  BKTS_API_BEGIN
  BKTS_REQUIRE(st, "stepper must not be NULL");
  BKTS_REQUIRE(n_steps >= 0, "n_steps must be >= 0");
  BKTS_REQUIRE(inner, "inner options must not be NULL");
  BKTS_REQUIRE(inner->rtol > 0.0 && inner->rtol < 1.0, "inner rtol must be in (0, 1)");
  BKTS_REQUIRE(outer_rtol > 0.0 && outer_rtol < 1.0, "outer_rtol must be in (0, 1)");
  BKTS_REQUIRE(max_outer >= 1, "max_outer must be >= 1");
  set_device(st->ctx);
  return st->advance(n_steps, *inner, outer_rtol, max_outer, y_hist, cb, user, info);
  BKTS_API_END
}

bkts_status bkts_stepper_state(bkts_stepper st, double* y, int64_t* accepted) {
  BKTS_API_BEGIN
  BKTS_REQUIRE(st, "stepper must not be NULL");
  set_device(st->ctx);
  if (y)
    BKTS_HIP(hipMemcpyAsync(y, st->yprev.p, sizeof(double) * st->op->N, hipMemcpyDeviceToDevice, st->ctx->stream));
  st->ctx->sync();
  if (accepted) *accepted = st->accepted;
  BKTS_API_END
}

bkts_status bkts_nlop_create(bkts_ctx ctx, const bkts_grid* grid, const bkts_nl_coeffs* coeffs, bkts_nlop* out) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  BKTS_REQUIRE(out, "out must not be NULL");
  *out = nullptr;
  set_device(ctx);
  *out = bkts::nlop_create(ctx, grid, coeffs);
  BKTS_API_END
}

bkts_status bkts_richards_create(bkts_ctx ctx, const bkts_grid* grid, const double* ks,
                                 const bkts_richards_params* params, bkts_nlop* out) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  BKTS_REQUIRE(out, "out must not be NULL");
  *out = nullptr;
  set_device(ctx);
  *out = bkts::richards_create(ctx, grid, ks, params);
  BKTS_API_END
}

bkts_status bkts_nl_mass(bkts_ctx ctx, bkts_nlop nl, int k, const double* Y, int ldy, double* M, int ldm) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  BKTS_REQUIRE(nl && nl->ctx == ctx, "nl must belong to ctx");
  check_k(k);
  check_block(Y, k, ldy, "Y");
  check_block(M, k, ldm, "M");
  set_device(ctx);
  bkts::nl_mass(ctx, *nl, k, Y, ldy, M, ldm);
  BKTS_API_END
}

void bkts_nlop_destroy(bkts_nlop nl) {
  if (!nl) return;
  (void)hipSetDevice(nl->ctx->device);
  (void)hipStreamSynchronize(nl->ctx->stream);
  delete nl;
}

bkts_status bkts_nl_eval(bkts_ctx ctx, bkts_nlop nl, int k, const double* Y, int ldy, double* F, int ldf) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  BKTS_REQUIRE(nl && nl->ctx == ctx, "nl must belong to ctx");
  check_k(k);
  check_block(Y, k, ldy, "Y");
  check_block(F, k, ldf, "F");
  BKTS_REQUIRE(Y != F, "Y and F must not alias");
  set_device(ctx);
  bkts::nl_eval(ctx, *nl, k, Y, ldy, F, ldf);
  BKTS_API_END
}

bkts_status bkts_nl_jacobian(bkts_ctx ctx, bkts_nlop nl, const double* u, double alpha, double beta, bkts_op* J) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  BKTS_REQUIRE(nl && nl->ctx == ctx, "nl must belong to ctx");
  BKTS_REQUIRE(u && J, "u and J must not be NULL");
  set_device(ctx);
  bkts::nl_jacobian(ctx, *nl, u, 1, alpha, beta);
  *J = nl->jac;
  BKTS_API_END
}

bkts_status bkts_nl_residual(bkts_ctx ctx, bkts_nlop nl, bkts_tc tc, int phase, const double* Y, int ldy,
                             const double* B0, int ldb0, int nb0, double* R, int ldr, double* col_norms2) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  BKTS_REQUIRE(nl && nl->ctx == ctx && tc, "nl must belong to ctx and tc must not be NULL");
  BKTS_REQUIRE(phase >= 0 && phase < tc->m_impl, "phase must be in 0..%d", tc->m_impl - 1);
  BKTS_REQUIRE(!tc->fully_implicit || phase == 0, "a fully implicit tableau's windows start at stage 0 (whole steps)");
  const int k = tc->k;
  check_block(Y, k, ldy, "Y");
  check_block(R, k, ldr, "R");
  BKTS_REQUIRE(Y != R, "Y and R must not alias");
  BKTS_REQUIRE(nb0 >= 0 && nb0 <= k && nb0 <= 8, "nb0 must be in 0..min(k, 8)");
  if (B0 && nb0 > 0) BKTS_REQUIRE(ldb0 >= nb0, "ldb0 < nb0");
  set_device(ctx);
  double* mats = ctx->ws.get<double>("api_nl_mats", 2 * k * k + k);
  double* nrm = ctx->ws.get<double>("api_res_nrm", k);
  bkts::upload_window(ctx, *tc, phase, 0, mats, mats + k * k, mats + 2 * k * k);
  int cols[8];
  for (int i = 0; i < 8; ++i) cols[i] = i;
  bkts::nl_residual(ctx, *nl, k, Y, ldy, mats, mats + k * k, B0, ldb0, B0 ? nb0 : 0, cols, R, ldr, nrm);
  if (col_norms2) {
    BKTS_HIP(hipMemcpyAsync(col_norms2, nrm, sizeof(double) * k, hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
  }
  BKTS_API_END
}

bkts_status bkts_newton_step(bkts_ctx ctx, bkts_nlop nl, bkts_tc tc, int phase, const double* B0, int ldb0, int nb0,
                             double* Y, double* col_norms2, const bkts_solve_opts* opts, bkts_solve_info* info) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  BKTS_REQUIRE(nl && nl->ctx == ctx && tc, "nl must belong to ctx and tc must not be NULL");
  BKTS_REQUIRE(phase >= 0 && phase < tc->m_impl, "phase must be in 0..%d", tc->m_impl - 1);
  BKTS_REQUIRE(!tc->fully_implicit || phase == 0, "a fully implicit tableau's windows start at stage 0 (whole steps)");
  BKTS_REQUIRE(Y && opts, "Y and opts must not be NULL");
  BKTS_REQUIRE(opts->rtol > 0.0 && opts->rtol < 1.0, "rtol must be in (0, 1)");
  const int k = tc->k;
  BKTS_REQUIRE(nb0 >= 0 && nb0 <= k && nb0 <= 8, "nb0 must be in 0..min(k, 8)");
  if (B0 && nb0 > 0) BKTS_REQUIRE(ldb0 >= nb0, "ldb0 < nb0");
  set_device(ctx);
  const int64_t N = nl->N;
  double* mats = ctx->ws.get<double>("api_nl_mats", 2 * k * k + k);
  double* nrm = ctx->ws.get<double>("api_res_nrm", k);
  double* R = ctx->ws.get<double>("api_newton_R", (size_t)N * k);
  double* V = ctx->ws.get<double>("api_newton_V", (size_t)N * k);
  bkts::upload_window(ctx, *tc, phase, 0, mats, mats + k * k, mats + 2 * k * k);
  int cols[8];
  for (int i = 0; i < 8; ++i) cols[i] = i;
  bkts::nl_residual(ctx, *nl, k, Y, k, mats, mats + k * k, B0, ldb0, B0 ? nb0 : 0, cols, R, k, nrm);
  if (col_norms2) BKTS_HIP(hipMemcpyAsync(col_norms2, nrm, sizeof(double) * k, hipMemcpyDeviceToHost, ctx->stream));
  bkts::nl_jacobian(ctx, *nl, Y, k, 1.0 / tc->tau, tc_beta(*tc, phase));
  bkts::KrylovStats st;
  bkts::solve(ctx, *nl->jac, 0.0, 1.0, k, R, V, true, *opts, false, st);
  bkts::axpby(ctx, N * k, -1.0, V, 1.0, Y);
  ctx->sync();
  if (info) {
    info->iterations = st.iterations;
    info->refinements = st.refinements;
    info->converged = st.converged;
    info->deflations = st.deflations;
    info->max_rel_residual = st.max_rel;
  }
  BKTS_API_END
}

bkts_status bkts_nl_stepper_create(bkts_ctx ctx, bkts_nlop nl, bkts_tc tc, const double* y0, bkts_stepper* out) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  BKTS_REQUIRE(out, "out must not be NULL");
  *out = nullptr;
  BKTS_REQUIRE(nl && nl->ctx == ctx && tc, "nl must belong to ctx and tc must not be NULL");
  BKTS_REQUIRE(y0, "y0 must not be NULL");
  BKTS_REQUIRE(!tc->fully_implicit, "the Newton stepper takes DIRK tableaux (lower triangular A)");
  set_device(ctx);
  *out = new bkts_stepper_s(ctx, nl->jac, tc, y0, nl);
  BKTS_API_END
}

void bkts_stepper_destroy(bkts_stepper st) {
  if (!st) return;
  (void)hipSetDevice(st->ctx->device);
  (void)hipStreamSynchronize(st->ctx->stream);
  delete st;
}


bkts_status bkts_server_create(bkts_ctx ctx, size_t hbm_budget_bytes, int max_slots, bkts_server* out) {
  BKTS_API_BEGIN
  check_ctx(ctx);
  BKTS_REQUIRE(out, "out must not be NULL");
  *out = nullptr;
  BKTS_REQUIRE(max_slots >= 1 && max_slots <= 256, "max_slots must be in 1..256");
  BKTS_REQUIRE(hbm_budget_bytes > 0, "hbm_budget_bytes must be > 0");
  set_device(ctx);
  *out = new bkts_server_s(ctx->device, hbm_budget_bytes, max_slots);
  BKTS_API_END
}

bkts_status bkts_server_submit(bkts_server srv, const bkts_request* req, uint64_t* ticket) {
  BKTS_API_BEGIN
  BKTS_REQUIRE(srv && req, "srv and req must not be NULL");
  const uint64_t t = srv->submit(*req);
  if (ticket) *ticket = t;
  BKTS_API_END
}

bkts_status bkts_server_poll(bkts_server srv, bkts_result* out, int max, int* n_done) {
  BKTS_API_BEGIN
  BKTS_REQUIRE(srv && n_done, "srv and n_done must not be NULL");
  BKTS_REQUIRE(max >= 0 && (out || max == 0), "out must hold max results");
  *n_done = srv->poll(out, max);
  {
    std::lock_guard<std::mutex> g(srv->mu);
    if (srv->fatal && *n_done == 0) throw Error{BKTS_EDEVICE, "server stopped: " + srv->fatal_msg};
  }
  BKTS_API_END
}

bkts_status bkts_server_wait(bkts_server srv, int n, double timeout_s, int* n_ready) {
  BKTS_API_BEGIN
  BKTS_REQUIRE(srv, "srv must not be NULL");
  const int r = srv->wait(n, timeout_s);
  if (n_ready) *n_ready = r;
  BKTS_API_END
}

bkts_status bkts_server_stats_get(bkts_server srv, bkts_server_stats* out) {
  BKTS_API_BEGIN
  BKTS_REQUIRE(srv && out, "srv and out must not be NULL");
  *out = srv->stats();
  BKTS_API_END
}

double bkts_server_clock(bkts_server srv) { return srv ? srv->now() : 0.0; }

void bkts_server_destroy(bkts_server srv) { delete srv; }

}  // extern "C"
